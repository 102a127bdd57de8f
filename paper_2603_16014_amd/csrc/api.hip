// C ABI of the fast MTGP library: plan construction, workspace layout and
// the orchestration of the device passes for each entry point.
//
// Evaluation order of one loss + gradient (equal sample sizes):
//   prep      decode theta -> Params (R = B B^T + diag zeta, exp of logs)
//   gen+A     kernel columns c_p regenerated from the design and transformed
//             over the low index bits in LDS (Eq. prod_kernel; Theorem
//             "Fast MTGP computations", item 3: lambda = transform of the
//             zeroth column of each pair block)
//   B         remaining high index bits
//   solve     per-frequency T x T Cholesky, log det, quadratic form, W
//   B^T, A^T  the adjoint transform of the weights, fused with the
//             derivative reduction over the regenerated columns
//   finalize  deterministic sums of block partials, chain rule
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mtgp.h"
#include "kernels.h"

using namespace mtgp;

#define MTGP_NPHASE 7
static const char* kPhaseNames[MTGP_NPHASE] = {"prep",  "gen_fwd_low",    "fwd_high", "solve",
                                               "adj_high", "adj_low_reduce", "finalize"};

struct mtgp_plan {
  int T, d, family, order, adaptive, s, profile, precision;
  int m[MTGP_MAXT];
  int64_t n[MTGP_MAXT];
  int64_t off[MTGP_MAXT + 1];
  int64_t N;
  bool equal;
  std::vector<uint32_t> gen;    // [d][32] (DSEQ) or [d] (LAT)
  std::vector<uint32_t> shift;  // [T][d]
  // distinct kernel columns, ordered by non-increasing length
  int ncol;
  std::vector<int> col_m, col_t, col_u;
  std::vector<int64_t> col_off;
  std::vector<uint32_t> col_shift;  // [ncol][d]
  PairMap pm;
  struct Group {
    int first, count, m;
  };
  std::vector<Group> groups;
  // device tables
  uint32_t* d_gen = nullptr;
  uint32_t* d_colshift = nullptr;
  ColInfo* d_colinfo = nullptr;  // per column: task pair, rows of the adjoint partial table
  uint32_t* d_taskshift = nullptr;
  // workspace layout (byte offsets)
  size_t o_params, o_status, o_cols, o_work, o_yhat, o_yh32, o_ahat, o_sp, o_sp2, o_ap, o_ap2,
      o_alpha, o_pwork, o_a1a, o_a1b, o_logs, o_lp2, o_misc, ws_bytes;
  int nadj_blocks;
  int64_t cols_elems;
  size_t real_bytes;  // bytes of a stored spectrum / adjoint value
  size_t work_bytes;  // bytes of a forward working value (0: works in the spectrum buffer)
  Sched sched;
  Alg1Desc a1;      // stage descriptors of the unequal-size elimination
  int64_t a1_ms;    // final block size N / n_T
  int elim = MTGP_ELIM_SPARSE;  // unequal sizes: fill-free LDL^H or Algorithm 1
  // optional phase timing (profiling aid; not thread safe)
  // Overlap of the VALU-bound fused passes (caller's stream) with the
  // HBM-bound strided passes (aux stream) over chunks of columns; fork and
  // join through events, so the sequence can be captured in a HIP graph.
  // Events are re-recorded round-robin: a wait takes the event's state at the
  // time it is enqueued, so reuse after the matching wait is safe.  Each
  // record and its wait are taken together under a lock, so calls on one
  // plan from several host threads never re-record an event between another
  // call's record and wait.
  static constexpr int kMaxChunks = 32;
  static constexpr int kEvents = 32;
  int nchunks = 4;
  hipStream_t aux = nullptr;
  hipEvent_t xev[kEvents] = {};
  mutable std::mutex xev_lock;
  mutable int xev_next = 0;
  // makes `to` wait for the work enqueued so far on `from`
  hipError_t fork(hipStream_t from, hipStream_t to) const {
    std::lock_guard<std::mutex> g(xev_lock);
    const hipEvent_t e = xev[xev_next];
    xev_next = (xev_next + 1) % kEvents;
    hipError_t r = hipEventRecord(e, from);
    if (r == hipSuccess) r = hipStreamWaitEvent(to, e, 0);
    return r;
  }
  // a ring of event sets lets many calls be timed without a host wait
  static constexpr int kRing = 64;
  bool timing = false;
  int ev_slot = 0;     // set the next call records into
  int ev_pending = 0;  // calls recorded since the last mtgp_phase_times
  hipEvent_t ev[kRing][MTGP_NPHASE + 1] = {};
  KDesc kd() const {
    KDesc k;
    k.T = T;
    k.d = d;
    k.family = family;
    k.order = order;
    k.adaptive = adaptive;
    k.s = s;
    k.profile = profile;
    k.unequal = equal ? 0 : 1;
    k.gcv = 0;
    for (int t = 0; t < MTGP_MAXT; t++) k.m[t] = t < T ? m[t] : 0;
    return k;
  }
};

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

#define HIP_OK(expr)                        \
  do {                                      \
    if ((expr) != hipSuccess) return MTGP_EHIP; \
  } while (0)
#define LAUNCH_OK(...)                        \
  do {                                        \
    if ((__VA_ARGS__) != 0) return MTGP_EHIP; \
  } while (0)

struct WsView {
  Params* P;
  int* status;
  unsigned char* cols;
  unsigned char* work;
  double* yhat;
  float* yh32;  // FP32 copy of yhat for the equal-size solves of FP32-stored spectra
  double* ahat;
  double* sp;
  double* sp2;
  double* ap;
  double* ap2;
  double* alpha;
  double* pwork;
  z2* a1a;
  z2* a1b;
  double* logs;
  double* lp2;
  double* misc;
};

WsView view(const mtgp_plan* p, void* ws) {
  unsigned char* b = static_cast<unsigned char*>(ws);
  WsView v;
  v.P = reinterpret_cast<Params*>(b + p->o_params);
  v.status = reinterpret_cast<int*>(b + p->o_status);
  v.cols = b + p->o_cols;
  v.work = p->work_bytes ? b + p->o_work : b + p->o_cols;
  v.yhat = reinterpret_cast<double*>(b + p->o_yhat);
  v.yh32 = reinterpret_cast<float*>(b + p->o_yh32);
  v.ahat = reinterpret_cast<double*>(b + p->o_ahat);
  v.sp = reinterpret_cast<double*>(b + p->o_sp);
  v.sp2 = reinterpret_cast<double*>(b + p->o_sp2);
  v.ap = reinterpret_cast<double*>(b + p->o_ap);
  v.ap2 = reinterpret_cast<double*>(b + p->o_ap2);
  v.alpha = reinterpret_cast<double*>(b + p->o_alpha);
  v.pwork = reinterpret_cast<double*>(b + p->o_pwork);
  v.a1a = reinterpret_cast<z2*>(b + p->o_a1a);
  v.a1b = reinterpret_cast<z2*>(b + p->o_a1b);
  v.logs = reinterpret_cast<double*>(b + p->o_logs);
  v.lp2 = reinterpret_cast<double*>(b + p->o_lp2);
  v.misc = reinterpret_cast<double*>(b + p->o_misc);
  return v;
}

int64_t theta_size(const mtgp_plan* p) {
  return (int64_t)p->T + 1 + p->d + (p->adaptive ? 4 : 0) + p->T + (int64_t)p->T * p->s + p->T;
}

inline void mark(const mtgp_plan* p, int phase, hipStream_t st) {
  if (p->timing) (void)hipEventRecord(p->ev[p->ev_slot][phase], st);
}

// closes the event set of one timed call
inline void mark_done(const mtgp_plan* p, hipStream_t st) {
  if (!p->timing) return;
  mtgp_plan* q = const_cast<mtgp_plan*>(p);
  (void)hipEventRecord(q->ev[q->ev_slot][MTGP_NPHASE], st);
  q->ev_slot = (q->ev_slot + 1) % mtgp_plan::kRing;
  q->ev_pending = std::min(q->ev_pending + 1, mtgp_plan::kRing);
}

// Whether the caller's stream is being captured into a HIP graph.  The
// overlapped passes fork onto the plan's own stream; under capture they are
// switched off and the passes run in order on the caller's stream (a capture
// of many fits forked from side streams ended in a host-side fault inside
// the runtime's capture end with the fork enabled; its cause is not known).
inline bool capturing(hipStream_t st) {
  hipStreamCaptureStatus s = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &s) == hipSuccess && s != hipStreamCaptureStatusNone;
}

// Column chunks of a group for the overlapped passes: [lo, hi) of chunk k.
inline void chunk_range(int first, int count, int nch, int k, int& lo, int& hi) {
  lo = first + (int)((int64_t)count * k / nch);
  hi = first + (int)((int64_t)count * (k + 1) / nch);
}

// Whether a digital-net group's adjoint keeps its working buffer in the run
// layout: only when the buffer is its own (not the weights') and the high
// bits are one 12-bit pass with 8 columns per block.  The one pass then
// writes every wave access as 512 contiguous values and the reduction reads
// whole lines (measured at 2^24 points: 1.92 -> 1.62 ms for the adjoint
// pass).  The forward keeps the natural layout: reading runs there made
// its one pass slower (1.70 -> 2.04 ms) whatever the XCD placement.
template <typename CR, typename SR>
int group_runs(const mtgp_plan* p, int m) {
  return p->work_bytes && strided_runs(p->sched, m, sizeof(CR), sizeof(SR), sizeof(CR)) ? 1 : 0;
}

// Kernel columns and their forward transforms: arithmetic in CR, spectrum
// stored as SR.  When CR != SR the working buffer holds the partially
// transformed columns and only the final pass rounds to SR.
template <typename CR, typename SR>
int run_columns(const mtgp_plan* p, const WsView& w, hipStream_t st) {
  SR* spec = reinterpret_cast<SR*>(w.cols);
  CR* work = reinterpret_cast<CR*>(w.work);
  const KDesc kd = p->kd();
  mark(p, 1, st);
  const bool ovl = p->aux && p->nchunks > 1 && !capturing(st);
  if (!ovl) {
    for (const auto& g : p->groups) {
      const int64_t len = (int64_t)1 << g.m;
      const uint32_t* sh = p->d_colshift + (size_t)g.first * p->d;
      if (g.m > p->sched.lb(g.m))
        LAUNCH_OK(launch_gen_fwd<CR, CR>(work + p->col_off[g.first], len, g.count, g.m, p->d_gen,
                                         sh, w.P, kd, p->sched, st));
      else
        LAUNCH_OK(launch_gen_fwd<CR, SR>(spec + p->col_off[g.first], len, g.count, g.m, p->d_gen,
                                         sh, w.P, kd, p->sched, st));
    }
    mark(p, 2, st);
    for (const auto& g : p->groups) {
      const int64_t o = p->col_off[g.first];
      LAUNCH_OK(launch_strided<CR, CR, SR>(work + o, work + o, spec + o, (int64_t)1 << g.m,
                                           g.count, g.m, p->sched, st));
    }
    return MTGP_OK;
  }
  // generation + low pass of chunk k on st, its high passes on aux once the
  // chunk is written; aux joins st before the solve
  HIP_OK(p->fork(st, p->aux));
  for (const auto& g : p->groups) {
    const int64_t len = (int64_t)1 << g.m;
    const bool high = g.m > p->sched.lb(g.m);
    const int nch = high ? std::min(p->nchunks, g.count) : 1;
    for (int k = 0; k < nch; k++) {
      int c0, c1;
      chunk_range(g.first, g.count, nch, k, c0, c1);
      const uint32_t* sh = p->d_colshift + (size_t)c0 * p->d;
      const int64_t o = p->col_off[c0];
      if (!high) {
        LAUNCH_OK(launch_gen_fwd<CR, SR>(spec + o, len, c1 - c0, g.m, p->d_gen, sh, w.P, kd,
                                         p->sched, st));
        continue;
      }
      LAUNCH_OK(launch_gen_fwd<CR, CR>(work + o, len, c1 - c0, g.m, p->d_gen, sh, w.P, kd,
                                       p->sched, st));
      HIP_OK(p->fork(st, p->aux));
      LAUNCH_OK(launch_strided<CR, CR, SR>(work + o, work + o, spec + o, len, c1 - c0, g.m,
                                           p->sched, p->aux));
    }
  }
  HIP_OK(p->fork(p->aux, st));
  mark(p, 2, st);
  return MTGP_OK;
}

// Forward transforms of all kernel columns (CR arithmetic, spectrum as SR).
template <typename CR, typename SR>
int forward_columns(const mtgp_plan* p, const WsView& w, hipStream_t st) {
  if (p->family == MTGP_DSEQ) return run_columns<CR, SR>(p, w, st);
  const KDesc kd = p->kd();
  cx<SR>* spec = reinterpret_cast<cx<SR>*>(w.cols);
  cx<CR>* work = reinterpret_cast<cx<CR>*>(w.work);
  mark(p, 1, st);
  for (const auto& g : p->groups) {
    const int64_t o = p->col_off[g.first];
    LAUNCH_OK(launch_lat_forward<CR, SR>(LAT_SRC_GEN, work + o, spec + o, (int64_t)1 << g.m,
                                         g.count, g.m, nullptr, 0, 1.0, p->d_gen,
                                         p->d_colshift + (size_t)g.first * p->d, w.P, kd, st));
  }
  mark(p, 2, st);
  return MTGP_OK;
}

// Adjoint high passes of digital-net columns, from the adjoint weights into
// the working buffer in the arithmetic's width.  (Storing these partial sums
// in the weights' FP32 width in the mixed mode was measured to move the
// gradient at T=8, d=10, n=2^24 by 3e-4 of its largest entry: the sums over
// the high bits mix the large low-frequency weights into every entry before
// the rounding.)  A group whose length fits the low pass has no high passes.
template <typename CR, typename SR>
int adj_high(const mtgp_plan* p, const SR* spec, CR* work, int64_t len, int ncols, int m,
             hipStream_t st) {
  if (m <= p->sched.lb(m)) return 0;
  return launch_strided<CR, SR, CR>(spec, work, work, len, ncols, m, p->sched, st,
                                    group_runs<CR, SR>(p, m));
}

// The low adjoint pass fused with the derivative reduction, reading where
// adj_high left the partially transformed weights.
template <typename CR, typename SR>
int adj_low(const mtgp_plan* p, const SR* spec, const CR* work, int64_t len, int ncols, int m,
            const uint32_t* sh, const Params* P, const KDesc& kd, double* part, hipStream_t st) {
  const Sched& sc = p->sched;
  if (m <= sc.lb(m))
    return launch_adj_reduce<CR, SR>(spec, len, ncols, m, p->d_gen, sh, P, kd, part, sc, st);
  return launch_adj_reduce<CR, CR>(work, len, ncols, m, p->d_gen, sh, P, kd, part, sc, st,
                                   group_runs<CR, SR>(p, m));
}

// Adjoint transforms of the weights fused with the derivative reduction;
// returns the number of partial rows written to w.ap (or a negative error).
template <typename CR, typename SR>
int adjoint_columns(const mtgp_plan* p, const WsView& w, hipStream_t st) {
  const KDesc kd = p->kd();
  int nadj = 0;
  if (p->family == MTGP_DSEQ) {
    SR* spec = reinterpret_cast<SR*>(w.cols);
    CR* work = reinterpret_cast<CR*>(w.work);
    const bool ovl = p->aux && p->nchunks > 1 && !capturing(st);
    if (!ovl) {
      for (const auto& g : p->groups) {
        const int64_t o = p->col_off[g.first];
        LAUNCH_OK(adj_high<CR, SR>(p, spec + o, work + o, (int64_t)1 << g.m, g.count, g.m, st));
      }
      mark(p, 5, st);
      for (const auto& g : p->groups) {
        const int64_t o = p->col_off[g.first];
        const int nb = (int)dseq_adj_rows(g.m, p->sched.lb(g.m));
        const uint32_t* sh = p->d_colshift + (size_t)g.first * p->d;
        double* part = w.ap + (size_t)nadj * adj_nq(p->d);
        LAUNCH_OK(adj_low<CR, SR>(p, spec + o, work + o, (int64_t)1 << g.m, g.count, g.m, sh, w.P,
                                  kd, part, st));
        nadj += nb * g.count;
      }
      return nadj;
    }
    // high passes of chunk k on aux, then its fused low pass + reduction on
    // st; partial rows keep the column order of the non-overlapped sequence
    HIP_OK(p->fork(st, p->aux));
    mark(p, 5, st);
    for (const auto& g : p->groups) {
      const int64_t len = (int64_t)1 << g.m;
      const int nb = (int)dseq_adj_rows(g.m, p->sched.lb(g.m));
      const bool high = g.m > p->sched.lb(g.m);
      const int nch = high ? std::min(p->nchunks, g.count) : 1;
      for (int k = 0; k < nch; k++) {
        int c0, c1;
        chunk_range(g.first, g.count, nch, k, c0, c1);
        const int64_t o = p->col_off[c0];
        const uint32_t* sh = p->d_colshift + (size_t)c0 * p->d;
        double* part = w.ap + (size_t)(nadj + (c0 - g.first) * nb) * adj_nq(p->d);
        if (!high) {
          LAUNCH_OK(launch_adj_reduce<CR, SR>(spec + o, len, c1 - c0, g.m, p->d_gen, sh, w.P, kd,
                                              part, p->sched, st));
          continue;
        }
        LAUNCH_OK(adj_high<CR, SR>(p, spec + o, work + o, len, c1 - c0, g.m, p->aux));
        HIP_OK(p->fork(p->aux, st));
        LAUNCH_OK(adj_low<CR, SR>(p, spec + o, work + o, len, c1 - c0, g.m, sh, w.P, kd, part,
                                  st));
      }
      nadj += nb * g.count;
    }
    // join aux back (its last chunk was already waited for; this covers
    // groups without high passes)
    HIP_OK(p->fork(p->aux, st));
    return nadj;
  }
  cx<SR>* spec = reinterpret_cast<cx<SR>*>(w.cols);
  cx<CR>* work = reinterpret_cast<cx<CR>*>(w.work);
  mark(p, 5, st);
  for (const auto& g : p->groups) {
    const int64_t o = p->col_off[g.first];
    LAUNCH_OK(launch_lat_adjoint<CR, SR>(LAT_SINK_REDUCE, spec + o, work + o, nullptr,
                                         (int64_t)1 << g.m, g.count, g.m, 0, 1.0, p->d_gen,
                                         p->d_colshift + (size_t)g.first * p->d, w.P, kd,
                                         w.ap + (size_t)nadj * adj_nq(p->d), st));
    nadj += lat_adj_blocks(g.m, sizeof(cx<CR>)) * g.count;
  }
  return nadj;
}

// Loss (and gradient): columns and transforms in CR arithmetic, spectrum and
// adjoint weights stored as SR, adjoint transform arithmetic in CR.  Equal
// sizes: per-frequency T x T factorisations; nested unequal sizes: the
// elimination in task order.
template <typename CR, typename SR>
int run_loss(const mtgp_plan* p, const double* theta, double* out3, double* grad, double* tau_hat,
             void* ws, hipStream_t st, bool want_ahat) {
  const WsView w = view(p, ws);
  const KDesc kd = p->kd();
  mark(p, 0, st);
  LAUNCH_OK(launch_prep(theta, w.P, kd, w.status, st));
  int rc = forward_columns<CR, SR>(p, w, st);
  if (rc) return rc;
  SR* spec = reinterpret_cast<SR*>(w.cols);
  const int64_t n = p->n[0];
  int64_t nsolve;
  mark(p, 3, st);
  if (!p->equal && p->elim == MTGP_ELIM_ALG1) {
    LAUNCH_OK(launch_alg1<SR>(spec, p->a1, w.P, kd.family, grad != nullptr, w.yhat, w.a1a, w.a1b,
                              w.logs, want_ahat ? w.ahat : nullptr, w.sp, w.status, st));
    nsolve = p->n[p->T - 1];
  } else if (!p->equal) {
    LAUNCH_OK(launch_zerofill<SR>(spec, p->a1, p->N, w.P, kd.family, grad != nullptr, w.yhat,
                                  w.a1a, w.logs, want_ahat ? w.ahat : nullptr, w.sp, w.status,
                                  st));
    nsolve = zf_final_blocks(p->N);
  } else if (p->family == MTGP_LAT) {
    LAUNCH_OK(launch_solve_eq_c<SR>(spec, n, p->pm, solve_yhat<SR>(w), w.yhat, w.P, kd,
                                    grad != nullptr, w.sp, want_ahat ? w.ahat : nullptr,
                                    w.status, st));
    nsolve = solve_blocks(n);
  } else {
    LAUNCH_OK(launch_solve_eq<SR>(spec, n, p->pm, p->ncol, solve_yhat<SR>(w), w.yhat, w.P, kd,
                                  grad != nullptr, w.sp, want_ahat ? w.ahat : nullptr, w.status,
                                  st));
    nsolve = solve_blocks(n);
  }
  mark(p, 4, st);
  int nadj = 0;
  if (grad) {
    nadj = adjoint_columns<CR, SR>(p, w, st);
    if (nadj < 0) return nadj;
  } else {
    mark(p, 5, st);
  }
  mark(p, 6, st);
  if (grad) {
    if (nadj != p->nadj_blocks) return MTGP_EINVAL;  // table rows must match the column map
    LAUNCH_OK(launch_colseg(w.ap, p->d_colinfo, p->ncol, adj_nq(p->d), w.ap2, st));
  }
  LAUNCH_OK(launch_colsum(w.sp, nsolve, solve_ns(p->T), w.sp2, COLSUM_BLOCKS, st));
  if (!p->equal) LAUNCH_OK(launch_colsum(w.logs, p->N, 1, w.lp2, COLSUM_BLOCKS, st));
  LAUNCH_OK(launch_finalize(w.sp2, COLSUM_BLOCKS, grad ? w.ap2 : nullptr, p->d_colinfo, p->ncol,
                            p->equal ? nullptr : w.lp2, COLSUM_BLOCKS, w.yhat, n, w.P, kd, out3,
                            grad, tau_hat, st));
  mark_done(p, st);
  return MTGP_OK;
}

// GCV loss (and gradient) for equal sizes: pass 1 forms q and s, pass 2
// (gradient) the weights W that need them; the rest is the MLE pipeline.
template <typename CR, typename SR>
int run_gcv(const mtgp_plan* p, const double* theta, double* out3, double* grad, double* tau_hat,
            void* ws, hipStream_t st) {
  const WsView w = view(p, ws);
  KDesc kd = p->kd();
  kd.gcv = 1;
  LAUNCH_OK(launch_prep(theta, w.P, kd, w.status, st));
  int rc = forward_columns<CR, SR>(p, w, st);
  if (rc) return rc;
  SR* spec = reinterpret_cast<SR*>(w.cols);
  const int64_t n = p->n[0];
  LAUNCH_OK(launch_gcv_eq<SR>(spec, n, p->pm, w.yhat, w.P, kd, false, w.sp, w.status, st));
  LAUNCH_OK(launch_colsum(w.sp, solve_blocks(n), solve_ns(p->T), w.sp2, COLSUM_BLOCKS, st));
  LAUNCH_OK(launch_finalize(w.sp2, COLSUM_BLOCKS, nullptr, p->d_colinfo, p->ncol, nullptr, 0,
                            w.yhat, n, w.P, kd, out3, nullptr, tau_hat, st));
  if (!grad) return MTGP_OK;
  LAUNCH_OK(launch_gcv_eq<SR>(spec, n, p->pm, w.yhat, w.P, kd, true, w.sp, w.status, st));
  const int nadj = adjoint_columns<CR, SR>(p, w, st);
  if (nadj < 0) return nadj;
  if (nadj != p->nadj_blocks) return MTGP_EINVAL;
  LAUNCH_OK(launch_colseg(w.ap, p->d_colinfo, p->ncol, adj_nq(p->d), w.ap2, st));
  LAUNCH_OK(launch_colsum(w.sp, solve_blocks(n), solve_ns(p->T), w.sp2, COLSUM_BLOCKS, st));
  LAUNCH_OK(launch_finalize(w.sp2, COLSUM_BLOCKS, w.ap2, p->d_colinfo, p->ncol, nullptr, 0,
                            w.yhat, n, w.P, kd, out3, grad, tau_hat, st));
  return MTGP_OK;
}

// GCV loss at nested sizes (no gradient): the fill-free elimination with
// the inverse's diagonal, GCV means from residue class 0.
template <typename CR, typename SR>
int run_gcv_nested(const mtgp_plan* p, const double* theta, double* out3, double* tau_hat,
                   void* ws, hipStream_t st) {
  const WsView w = view(p, ws);
  KDesc kd = p->kd();
  kd.gcv = 1;
  LAUNCH_OK(launch_prep(theta, w.P, kd, w.status, st));
  int rc = forward_columns<CR, SR>(p, w, st);
  if (rc) return rc;
  SR* spec = reinterpret_cast<SR*>(w.cols);
  LAUNCH_OK(launch_zerofill_gcv<SR>(spec, p->a1, p->N, w.P, kd.family, w.yhat, w.a1a, w.logs,
                                    w.sp, w.status, st));
  const int64_t nb = zf_final_blocks(p->N);
  LAUNCH_OK(launch_colsum(w.sp, nb, solve_ns(p->T), w.sp2, COLSUM_BLOCKS, st));
  LAUNCH_OK(launch_finalize(w.sp2, COLSUM_BLOCKS, nullptr, p->d_colinfo, p->ncol, nullptr, 0,
                            w.yhat, p->n[0], w.P, kd, out3, nullptr, tau_hat, st));
  return MTGP_OK;
}

// GCV loss and gradient at nested sizes: the elimination in dual numbers
// gives Lambda^-1 and Lambda^-2 on the pattern (and ahat, bhat), the first
// pass q and s, the second the weights of the adjoint.
template <typename CR, typename SR>
int run_gcv_nested_grad(const mtgp_plan* p, const double* theta, double* out3, double* grad,
                        double* tau_hat, void* ws, hipStream_t st) {
  const WsView w = view(p, ws);
  KDesc kd = p->kd();
  kd.gcv = 1;
  LAUNCH_OK(launch_prep(theta, w.P, kd, w.status, st));
  int rc = forward_columns<CR, SR>(p, w, st);
  if (rc) return rc;
  SR* spec = reinterpret_cast<SR*>(w.cols);
  const int64_t nb = zf_final_blocks(p->N);
  LAUNCH_OK(launch_zerofill_gcv_dual<SR>(spec, p->a1, p->N, w.P, kd.family, w.yhat, w.a1a, w.sp,
                                         w.status, false, st));
  LAUNCH_OK(launch_colsum(w.sp, nb, solve_ns(p->T), w.sp2, COLSUM_BLOCKS, st));
  LAUNCH_OK(launch_finalize(w.sp2, COLSUM_BLOCKS, nullptr, p->d_colinfo, p->ncol, nullptr, 0,
                            w.yhat, p->n[0], w.P, kd, out3, nullptr, tau_hat, st));
  LAUNCH_OK(launch_zerofill_gcv_dual<SR>(spec, p->a1, p->N, w.P, kd.family, w.yhat, w.a1a, w.sp,
                                         w.status, true, st));
  const int nadj = adjoint_columns<CR, SR>(p, w, st);
  if (nadj < 0) return nadj;
  if (nadj != p->nadj_blocks) return MTGP_EINVAL;
  LAUNCH_OK(launch_colseg(w.ap, p->d_colinfo, p->ncol, adj_nq(p->d), w.ap2, st));
  LAUNCH_OK(launch_colsum(w.sp, nb, solve_ns(p->T), w.sp2, COLSUM_BLOCKS, st));
  LAUNCH_OK(launch_finalize(w.sp2, COLSUM_BLOCKS, w.ap2, p->d_colinfo, p->ncol, nullptr, 0,
                            w.yhat, p->n[0], w.P, kd, out3, grad, tau_hat, st));
  return MTGP_OK;
}

int dispatch_loss(const mtgp_plan* p, const double* theta, double* out3, double* grad,
                  double* tau_hat, void* ws, hipStream_t st, bool want_ahat) {
  switch (p->precision) {
    case MTGP_FP64: return run_loss<double, double>(p, theta, out3, grad, tau_hat, ws, st, want_ahat);
    case MTGP_MIXED: return run_loss<double, float>(p, theta, out3, grad, tau_hat, ws, st, want_ahat);
    default: return run_loss<float, float>(p, theta, out3, grad, tau_hat, ws, st, want_ahat);
  }
}

// Equal sizes with FP32 spectrum storage: the per-frequency solves read the
// data transform from an FP32 copy (rounded once from the FP64 transform,
// like the spectrum; frequency 0, from which the means are subtracted, is
// read in FP64), which moves 4 instead of 8 bytes per point and task.
bool solve_yh32(const mtgp_plan* p) { return p->equal && p->real_bytes == sizeof(float); }
template <typename SR>
const SR* solve_yhat(const WsView& w);
template <>
const double* solve_yhat<double>(const WsView& w) { return w.yhat; }
template <>
const float* solve_yhat<float>(const WsView& w) { return w.yh32; }

// Workspace layout; depends on the schedule through the number of blocks of
// the adjoint reduction.
void layout(mtgp_plan* p) {
  const int T = p->T, d = p->d;
  const size_t cplx = p->family == MTGP_LAT ? 2 : 1;
  size_t o = 0;
  p->o_params = o;
  o = align_up(o + sizeof(Params));
  p->o_status = o;
  o = align_up(o + 64);
  p->o_cols = o;
  o = align_up(o + (size_t)p->cols_elems * p->real_bytes * cplx);
  p->o_work = o;
  o = align_up(o + (size_t)p->cols_elems * p->work_bytes * cplx);
  p->o_yhat = o;
  o = align_up(o + (size_t)p->N * sizeof(double) * cplx);
  p->o_yh32 = o;
  o = align_up(o + (solve_yh32(p) ? (size_t)p->N * sizeof(float) * cplx : 0));
  p->o_ahat = o;
  o = align_up(o + (size_t)p->N * sizeof(double) * cplx);
  p->o_alpha = o;
  o = align_up(o + (cplx == 2 ? (size_t)p->N * sizeof(double) : 0));
  p->o_pwork = o;
  o = align_up(o + (cplx == 2 ? (size_t)p->N * 2 * sizeof(double) : 0));
  // unequal sizes: Algorithm 1 keeps two running-inverse buffers of N m_T
  // entries; the fill-free elimination one buffer of pattern values and
  // right-hand sides
  const bool a1dense = !p->equal && p->elim == MTGP_ELIM_ALG1;
  const size_t a1 = a1dense ? (size_t)p->N * (size_t)p->a1_ms * sizeof(z2) : 0;
  // (pairs of complex values: the GCV gradient runs the elimination in dual numbers)
  const size_t zf = !p->equal && !a1dense ? (size_t)zf_elems(p->a1, p->N) * 2 * sizeof(z2) : 0;
  p->o_a1a = o;
  o = align_up(o + (a1dense ? a1 : zf));
  p->o_a1b = o;
  o = align_up(o + a1);
  p->o_logs = o;
  o = align_up(o + (p->equal ? 0 : (size_t)p->N * sizeof(double)));
  p->o_lp2 = o;
  o = align_up(o + (size_t)COLSUM_BLOCKS * sizeof(double));
  p->o_sp = o;
  {
    const int64_t rows = p->equal ? solve_blocks(p->n[0])
                                  : std::max<int64_t>(p->n[p->T - 1], zf_final_blocks(p->N));
    o = align_up(o + (size_t)rows * solve_ns(T) * sizeof(double));
  }
  p->o_sp2 = o;
  o = align_up(o + (size_t)COLSUM_BLOCKS * solve_ns(T) * sizeof(double));
  p->nadj_blocks = 0;
  for (const auto& g : p->groups) {
    if (p->family == MTGP_LAT)
      p->nadj_blocks += lat_adj_blocks(g.m, p->precision == MTGP_F32 ? sizeof(cx<float>)
                                                                      : sizeof(cx<double>)) *
                        g.count;
    else
      p->nadj_blocks += dseq_adj_rows(g.m, p->sched.lb(g.m)) * g.count;
  }
  p->o_ap = o;
  o = align_up(o + (size_t)p->nadj_blocks * adj_nq(d) * sizeof(double));
  p->o_ap2 = o;
  o = align_up(o + (size_t)std::max(COLSUM_BLOCKS, p->ncol) * adj_nq(d) * sizeof(double));
  p->o_misc = o;
  o = align_up(o + 4096);
  p->ws_bytes = o;
}

// Column map of the adjoint partial table (rows in the order adjoint_columns
// writes them: groups in order, within a group column-major blocks).
int upload_colinfo(mtgp_plan* p) {
  std::vector<ColInfo> ci(p->ncol);
  int64_t row = 0;
  for (const auto& g : p->groups) {
    const int64_t nb =
        p->family == MTGP_LAT
            ? lat_adj_blocks(g.m, p->precision == MTGP_F32 ? sizeof(cx<float>) : sizeof(cx<double>))
            : dseq_adj_rows(g.m, p->sched.lb(g.m));
    for (int c = g.first; c < g.first + g.count; c++) {
      ci[c].t = p->col_t[c];
      ci[c].u = p->col_u[c];
      ci[c].row_off = row;
      ci[c].row_cnt = nb;
      row += nb;
    }
  }
  if (row != p->nadj_blocks) return MTGP_EINVAL;
  if (!p->d_colinfo && hipMalloc(&p->d_colinfo, ci.size() * sizeof(ColInfo)) != hipSuccess)
    return MTGP_ENOMEM;
  if (hipMemcpy(p->d_colinfo, ci.data(), ci.size() * sizeof(ColInfo), hipMemcpyHostToDevice) !=
      hipSuccess)
    return MTGP_EHIP;
  return MTGP_OK;
}

bool valid_family_order(const mtgp_design* d) {
  if (d->family == MTGP_DSEQ) return d->kernel_order >= 1 && d->kernel_order <= 4;
  if (d->family == MTGP_LAT) return d->kernel_order >= 1 && d->kernel_order <= 3 && !d->adaptive;
  return false;
}

// Forward DFT of real rows (mtgp_fft); `scratch` holds the bit-reversed
// spectrum of the multi-pass sizes and is unused (may be NULL) for the
// single-pass ones.
int fft_run(const void* x, void* X, void* scratch, int64_t batch, int32_t log2n, int32_t dtype,
            int32_t bitrev_input, hipStream_t st) {
  if (batch < 0 || batch > 65535 || log2n < 0 || log2n > 30) return MTGP_EINVAL;
  if (dtype != MTGP_DTYPE_F64 && dtype != MTGP_DTYPE_F32) return MTGP_EINVAL;
  if (batch == 0) return MTGP_OK;
  const bool single = lat_single_pass(log2n);
  if (!x || !X || (!single && !scratch)) return MTGP_EINVAL;
  const int src = bitrev_input ? LAT_SRC_Y : LAT_SRC_X;
  const int64_t n = (int64_t)1 << log2n;
  const int f32 = dtype == MTGP_DTYPE_F32;
  if (single) {
    // one LDS pass writes natural frequency order itself
    if (f32)
      LAUNCH_OK(launch_lat_single_natural<float>(src, x, 1, static_cast<cx<float>*>(X), (int)batch,
                                                 log2n, st));
    else
      LAUNCH_OK(launch_lat_single_natural<double>(src, x, 0, static_cast<cx<double>*>(X),
                                                  (int)batch, log2n, st));
    return MTGP_OK;
  }
  KDesc kd{};
  kd.family = FAM_LAT;
  kd.order = 1;
  // Multi-pass sizes run in groups of at most 128 MiB of complex values, each
  // group through all its passes before the next (the scratch reused from
  // its start), so that a group's intermediate stays in the 256 MB
  // memory-side cache between passes, as for the Walsh transform.
  const size_t cbytes = f32 ? sizeof(cx<float>) : sizeof(cx<double>);
  const int64_t grp = std::max<int64_t>(1, ((int64_t)128 << 20) / (n * (int64_t)cbytes));
  for (int64_t b0 = 0; b0 < batch; b0 += grp) {
    const int nb = (int)std::min<int64_t>(grp, batch - b0);
    const void* xg = static_cast<const unsigned char*>(x) + b0 * n * (int64_t)(cbytes / 2);
    void* Xg = static_cast<unsigned char*>(X) + b0 * n * (int64_t)cbytes;
    if (lat_natural_out(log2n)) {
      // passes in scratch (every entry written before it is read), the last
      // one writing natural frequency order into X
      if (f32)
        LAUNCH_OK(launch_lat_forward<float, float>(src, static_cast<cx<float>*>(scratch),
                                                   static_cast<cx<float>*>(Xg), n, nb, log2n, xg, 1,
                                                   1.0, nullptr, nullptr, nullptr, kd, st, 1));
      else
        LAUNCH_OK(launch_lat_forward<double, double>(src, static_cast<cx<double>*>(scratch),
                                                     static_cast<cx<double>*>(Xg), n, nb, log2n,
                                                     xg, 0, 1.0, nullptr, nullptr, nullptr, kd,
                                                     st, 1));
      continue;
    }
    // bit-reversed spectrum in scratch, then permuted into X
    if (f32)
      LAUNCH_OK(launch_lat_forward<float, float>(src, static_cast<cx<float>*>(scratch),
                                                 static_cast<cx<float>*>(scratch), n, nb, log2n,
                                                 xg, 1, 1.0, nullptr, nullptr, nullptr, kd, st));
    else
      LAUNCH_OK(launch_lat_forward<double, double>(src, static_cast<cx<double>*>(scratch),
                                                   static_cast<cx<double>*>(scratch), n, nb,
                                                   log2n, xg, 0, 1.0, nullptr, nullptr, nullptr,
                                                   kd, st));
    LAUNCH_OK(launch_lat_natural(scratch, f32, Xg, nb, log2n, st));
  }
  return MTGP_OK;
}

// Scratch of mtgp_fft_noalloc: one static device array, which every GPU
// the library runs on holds (its own copy at its own address) until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy (on the host it only stands for the symbol); it uses the device
// address that hipGetSymbolAddress returns, looked up once per device on
// that device's first call and kept in fft_scratch_dev.
__device__ __align__(256) static unsigned char fft_noalloc_scratch[MTGP_FFT_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex fft_scratch_lock;
void* fft_scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of fft_noalloc_scratch.
int fft_scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MTGP_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return MTGP_ENOTSUP;
  std::lock_guard<std::mutex> g(fft_scratch_lock);
  if (!fft_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(fft_noalloc_scratch)) != hipSuccess || !ptr)
      return MTGP_EHIP;
    fft_scratch_dev[dev] = ptr;
  }
  *out = fft_scratch_dev[dev];
  return MTGP_OK;
}

}  // namespace

extern "C" {

const char* mtgp_strerror(int code) {
  switch (code) {
    case MTGP_OK: return "ok";
    case MTGP_EINVAL: return "invalid argument";
    case MTGP_ENOTPD: return "Lambda is not positive definite (or not finite) at some frequency";
    case MTGP_EHIP: return "HIP runtime error";
    case MTGP_ENOMEM: return "out of memory";
    case MTGP_ENOTSUP: return "not supported by this build";
    case MTGP_ETOOBIG: return "input larger than the static scratch of an allocation-free entry point";
  }
  return "unknown error";
}

int mtgp_plan_create(const mtgp_design* des, int32_t precision, mtgp_plan** out) {
  if (!des || !out || !des->m || !des->gen || !des->shift) return MTGP_EINVAL;
  *out = nullptr;
  if (des->T < 1 || des->T > MTGP_MAXT || des->d < 1 || des->d > MTGP_MAXD) return MTGP_EINVAL;
  if (des->rank_s < 1 || des->rank_s > MTGP_MAXS) return MTGP_EINVAL;
  if (!valid_family_order(des)) return MTGP_EINVAL;
  if (precision != MTGP_FP64 && precision != MTGP_MIXED && precision != MTGP_F32) return MTGP_EINVAL;
  for (int t = 0; t < des->T; t++) {
    if (des->m[t] < 0 || des->m[t] > 30) return MTGP_EINVAL;
    if (t > 0 && des->m[t] > des->m[t - 1]) return MTGP_EINVAL;
  }
  if (des->family == MTGP_LAT)
    for (int j = 0; j < des->d; j++)
      if (!(des->gen[j] & 1u)) return MTGP_EINVAL;
  mtgp_plan* p = new (std::nothrow) mtgp_plan();
  if (!p) return MTGP_ENOMEM;
  p->T = des->T;
  p->d = des->d;
  p->family = des->family;
  p->order = des->kernel_order;
  p->adaptive = des->adaptive ? 1 : 0;
  p->s = des->rank_s;
  p->profile = des->profile_tau ? 1 : 0;
  p->precision = precision;
  p->off[0] = 0;
  p->equal = true;
  for (int t = 0; t < p->T; t++) {
    p->m[t] = des->m[t];
    p->n[t] = (int64_t)1 << des->m[t];
    p->off[t + 1] = p->off[t] + p->n[t];
    if (des->m[t] != des->m[0]) p->equal = false;
  }
  p->N = p->off[p->T];
  const int gl = des->family == MTGP_DSEQ ? 32 : 1;
  p->gen.assign(des->gen, des->gen + (size_t)gl * des->d);
  p->shift.assign(des->shift, des->shift + (size_t)des->T * des->d);
  const int T = p->T, d = p->d;
  if (!p->equal) {
    int64_t ms = 0;
    for (int t = 0; t < T; t++) ms += p->n[t] >> p->m[T - 1];
    p->a1_ms = ms;  // Algorithm 1 (optional) needs ms <= ALG1_MAX_BLOCK
  } else {
    p->a1_ms = 0;
  }
  // columns: one diagonal column per distinct length (shift 0; every diagonal
  // pair of tasks with that length uses it), one per task pair t < u (length
  // n_t, the larger task: the tall case); then ordered by non-increasing
  // length so equal-length columns form contiguous groups
  auto pair_shift = [&](int t, int u, int j) -> uint32_t {
    const uint32_t a0 = p->shift[(size_t)t * d + j], b0 = p->shift[(size_t)u * d + j];
    return p->family == MTGP_DSEQ ? (a0 ^ b0) : (uint32_t)(a0 - b0);
  };
  struct ColSpec {
    int m, t, u;
  };
  std::vector<ColSpec> specs;
  int diag_of_m[31];
  for (int q = 0; q < 31; q++) diag_of_m[q] = -1;
  for (int t = 0; t < T; t++)
    if (diag_of_m[p->m[t]] < 0) {
      diag_of_m[p->m[t]] = (int)specs.size();
      specs.push_back({p->m[t], t, t});
    }
  for (int t = 0; t < T; t++)
    for (int u = t + 1; u < T; u++) specs.push_back({p->m[t], t, u});
  std::vector<int> order(specs.size());
  for (size_t q = 0; q < order.size(); q++) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return specs[x].m > specs[y].m; });
  std::vector<int> newidx(specs.size());
  std::memset(&p->pm, 0, sizeof(p->pm));
  p->ncol = (int)specs.size();
  for (int c = 0; c < p->ncol; c++) {
    const ColSpec& cs = specs[order[c]];
    newidx[order[c]] = c;
    p->col_m.push_back(cs.m);
    p->col_t.push_back(cs.t);
    p->col_u.push_back(cs.u);
    for (int j = 0; j < d; j++) p->col_shift.push_back(cs.t == cs.u ? 0u : pair_shift(cs.t, cs.u, j));
  }
  for (int t = 0; t < T; t++) p->pm.col[t][t] = (uint8_t)newidx[diag_of_m[p->m[t]]];
  {
    int q = (int)std::count_if(specs.begin(), specs.end(), [](const ColSpec& c) { return c.t == c.u; });
    for (int t = 0; t < T; t++)
      for (int u = t + 1; u < T; u++, q++) p->pm.col[t][u] = p->pm.col[u][t] = (uint8_t)newidx[q];
  }
  p->col_off.resize(p->ncol);
  int64_t acc = 0;
  for (int c = 0; c < p->ncol; c++) {
    p->col_off[c] = acc;
    acc += (int64_t)1 << p->col_m[c];
  }
  p->cols_elems = acc;
  for (int c = 0; c < p->ncol;) {
    int e2 = c;
    while (e2 < p->ncol && p->col_m[e2] == p->col_m[c]) e2++;
    p->groups.push_back({c, e2 - c, p->col_m[c]});
    c = e2;
  }
  // elimination descriptors
  std::memset(&p->a1, 0, sizeof(p->a1));
  p->a1.T = T;
  p->a1.profile = p->profile;
  int64_t so = 0;
  for (int s = 0; s < T; s++) {
    p->a1.m[s] = p->m[s];
    int64_t msz = 0;
    for (int t = 0; t <= s; t++) msz += p->n[t] >> p->m[s];
    p->a1.msz[s] = msz;
    p->a1.stage_off[s] = so;
    so += p->n[s];
    p->a1.task_off[s] = p->off[s];
    int first = s;
    for (int t = 0; t < s; t++)
      if (p->m[t] == p->m[s]) {
        first = t;
        break;
      }
    p->a1.diag_first[s] = (uint8_t)first;
  }
  {
    int64_t po = 0, co = 0;
    for (int a = 0; a < T; a++) {
      p->a1.so[a] = po;
      po += (int64_t)(T - a) * p->n[a];
      p->a1.coff[a] = co;
      co += p->n[a] >> p->m[T - 1];
    }
    p->a1.so[T] = po;
  }
  for (int t = 0; t < T; t++)
    for (int u = 0; u < T; u++) p->a1.pair_col[t][u] = p->pm.col[t][u];
  // every pair must read back (as the kernels read it) the column it was given
  for (int t = 0; t < T; t++)
    for (int u = 0; u < T; u++) {
      const int c = p->pm.at(t, u);
      const int lo = t < u ? t : u, hi = t < u ? u : t;
      if (c < 0 || c >= p->ncol || c != p->a1.pc(t, u) || p->col_m[c] != p->m[lo] ||
          (lo != hi && (p->col_t[c] != lo || p->col_u[c] != hi)) ||
          (lo == hi && p->col_t[c] != p->col_u[c])) {
        mtgp_plan_destroy(p);
        return MTGP_EINVAL;
      }
    }
  for (int c = 0; c < p->ncol; c++) {
    p->a1.col_m[c] = p->col_m[c];
    p->a1.col_off[c] = p->col_off[c];
  }
  p->real_bytes = precision == MTGP_FP64 ? sizeof(double) : sizeof(float);
  p->work_bytes = precision == MTGP_MIXED ? sizeof(double) : 0;
  layout(p);
  // device tables; digital sequences append the Gray-code step table of the
  // fused kernels (row k: z_j(256 gray(k)), the XOR of generating columns
  // 8 + b of dimension j over the set bits b of gray(k); zero beyond d)
  std::vector<uint32_t> genx = p->gen;
  if (p->family == MTGP_DSEQ) {
    genx.resize((size_t)32 * p->d + (size_t)GRAY_ROWS * GRAY_STRIDE, 0u);
    uint32_t* gz = genx.data() + (size_t)32 * p->d;
    for (int k = 0; k < GRAY_ROWS; k++) {
      const uint32_t gk = (uint32_t)(k ^ (k >> 1));
      for (int j = 0; j < p->d; j++) {
        uint32_t z = 0;
        for (int b = 0; b < 5; b++)
          if ((gk >> b) & 1u) z ^= p->gen[(size_t)32 * j + 8 + b];
        gz[(size_t)GRAY_STRIDE * k + j] = z;
      }
    }
  }
  if (hipMalloc(&p->d_gen, genx.size() * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&p->d_colshift, p->col_shift.size() * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&p->d_taskshift, p->shift.size() * sizeof(uint32_t)) != hipSuccess) {
    mtgp_plan_destroy(p);
    return MTGP_ENOMEM;
  }
  if (hipMemcpy(p->d_gen, genx.data(), genx.size() * sizeof(uint32_t),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_colshift, p->col_shift.data(), p->col_shift.size() * sizeof(uint32_t),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_taskshift, p->shift.data(), p->shift.size() * sizeof(uint32_t),
                hipMemcpyHostToDevice) != hipSuccess) {
    mtgp_plan_destroy(p);
    return MTGP_EHIP;
  }
  int rc = upload_colinfo(p);
  if (rc == MTGP_OK && p->family == MTGP_DSEQ) {
    // default priority, non-blocking with respect to the null stream
    if (hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking) != hipSuccess) rc = MTGP_EHIP;
    for (int k = 0; rc == MTGP_OK && k < mtgp_plan::kEvents; k++)
      if (hipEventCreateWithFlags(&p->xev[k], hipEventDisableTiming) != hipSuccess) rc = MTGP_EHIP;
  }
  if (rc != MTGP_OK) {
    mtgp_plan_destroy(p);
    return rc;
  }
  *out = p;
  return MTGP_OK;
}

int mtgp_plan_set_schedule(mtgp_plan* p, int32_t pass_a_bits, int32_t pass_b_bits,
                           int64_t pass_b_tile_bytes) {
  if (!p || pass_a_bits < 1 || pass_a_bits > PASS_A_MAX_BITS || pass_b_bits < 0 ||
      pass_b_bits > 12 || pass_b_tile_bytes < 4096 || pass_b_tile_bytes > 147456)
    return MTGP_EINVAL;
  p->sched.a_bits = pass_a_bits;
  p->sched.b_bits = pass_b_bits;
  p->sched.b_tile = (size_t)pass_b_tile_bytes;
  layout(p);
  return upload_colinfo(p);
}

int mtgp_plan_set_fused_occupancy(mtgp_plan* p, int32_t blocks_per_cu) {
  if (!p || blocks_per_cu < 0 || blocks_per_cu > 8) return MTGP_EINVAL;
  p->sched.fused_cap = blocks_per_cu;
  return MTGP_OK;
}

int mtgp_plan_set_elimination(mtgp_plan* p, int32_t mode) {
  if (!p || (mode != MTGP_ELIM_SPARSE && mode != MTGP_ELIM_ALG1)) return MTGP_EINVAL;
  if (mode == MTGP_ELIM_ALG1 && !p->equal && p->a1_ms > ALG1_MAX_BLOCK) return MTGP_ENOTSUP;
  p->elim = mode;
  layout(p);
  return MTGP_OK;
}

int mtgp_plan_set_overlap(mtgp_plan* p, int32_t chunks) {
  if (!p || chunks < 1 || chunks > mtgp_plan::kMaxChunks) return MTGP_EINVAL;
  p->nchunks = chunks;
  return MTGP_OK;
}

int mtgp_plan_enable_timing(mtgp_plan* p, int32_t on) {
  if (!p) return MTGP_EINVAL;
  if (on && !p->ev[0][0]) {
    for (int s = 0; s < mtgp_plan::kRing; s++)
      for (int k = 0; k <= MTGP_NPHASE; k++)
        if (hipEventCreate(&p->ev[s][k]) != hipSuccess) return MTGP_EHIP;
  }
  p->timing = on != 0;
  p->ev_pending = 0;
  return MTGP_OK;
}

int mtgp_phase_times(const mtgp_plan* p, double* ms, int32_t max_phases, int32_t* nphases) {
  if (!p || !p->ev[0][0] || (max_phases > 0 && !ms)) return MTGP_EINVAL;
  if (nphases) *nphases = MTGP_NPHASE;
  const int cnt = p->ev_pending;
  for (int k = 0; k < max_phases; k++) ms[k] = 0.0;
  if (cnt == 0) return MTGP_OK;
  const int last = (p->ev_slot + mtgp_plan::kRing - 1) % mtgp_plan::kRing;
  if (hipEventSynchronize(p->ev[last][MTGP_NPHASE]) != hipSuccess) return MTGP_EHIP;
  for (int c = 0; c < cnt; c++) {
    const int s = (p->ev_slot + mtgp_plan::kRing - 1 - c) % mtgp_plan::kRing;
    for (int k = 0; k < MTGP_NPHASE && k < max_phases; k++) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p->ev[s][k], p->ev[s][k + 1]) != hipSuccess) return MTGP_EHIP;
      ms[k] += t / cnt;
    }
  }
  const_cast<mtgp_plan*>(p)->ev_pending = 0;
  return MTGP_OK;
}

const char* mtgp_phase_name(int32_t k) {
  return (k >= 0 && k < MTGP_NPHASE) ? kPhaseNames[k] : "";
}

int mtgp_plan_destroy(mtgp_plan* p) {
  if (!p) return MTGP_OK;
  for (int s = 0; s < mtgp_plan::kRing; s++)
    for (int k = 0; k <= MTGP_NPHASE; k++)
      if (p->ev[s][k]) (void)hipEventDestroy(p->ev[s][k]);
  if (p->d_gen) (void)hipFree(p->d_gen);
  if (p->d_colshift) (void)hipFree(p->d_colshift);
  if (p->d_colinfo) (void)hipFree(p->d_colinfo);
  for (int k = 0; k < mtgp_plan::kEvents; k++)
    if (p->xev[k]) (void)hipEventDestroy(p->xev[k]);
  if (p->aux) (void)hipStreamDestroy(p->aux);
  if (p->d_taskshift) (void)hipFree(p->d_taskshift);
  delete p;
  return MTGP_OK;
}

int64_t mtgp_theta_size(const mtgp_plan* p) { return p ? theta_size(p) : MTGP_EINVAL; }
size_t mtgp_workspace_bytes(const mtgp_plan* p) { return p ? p->ws_bytes : 0; }
int64_t mtgp_num_points(const mtgp_plan* p) { return p ? p->N : MTGP_EINVAL; }
int32_t mtgp_num_columns(const mtgp_plan* p) { return p ? p->ncol : MTGP_EINVAL; }

int mtgp_column_info(const mtgp_plan* p, int32_t c, int32_t* log2n, int64_t* offset, int32_t* t,
                     int32_t* u) {
  if (!p || c < 0 || c >= p->ncol) return MTGP_EINVAL;
  if (log2n) *log2n = p->col_m[c];
  if (offset) *offset = p->col_off[c];
  if (t) *t = p->col_t[c];
  if (u) *u = p->col_u[c];
  return MTGP_OK;
}

int mtgp_gen_points(const mtgp_plan* p, int32_t task, int64_t first, int64_t count, uint32_t* out,
                    void* stream) {
  if (!p || task < 0 || task >= p->T || first < 0 || count < 0 || (count > 0 && !out))
    return MTGP_EINVAL;
  if (first + count > ((int64_t)1 << 32)) return MTGP_EINVAL;
  LAUNCH_OK(launch_gen_points(p->d_gen, p->d_taskshift + (size_t)task * p->d, p->family, p->d,
                              p->m[task], first, count, out, (hipStream_t)stream));
  return MTGP_OK;
}

int mtgp_kernel_cols(const mtgp_plan* p, const double* theta, void* cols, void* ws, void* stream) {
  if (!p || !theta || !cols || !ws) return MTGP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const WsView w = view(p, ws);
  const KDesc kd = p->kd();
  LAUNCH_OK(launch_prep(theta, w.P, kd, w.status, st));
  for (const auto& g : p->groups) {
    const uint32_t* sh = p->d_colshift + (size_t)g.first * p->d;
    if (p->precision != MTGP_F32)
      LAUNCH_OK(launch_raw_cols<double>(static_cast<double*>(cols) + p->col_off[g.first], g.count,
                                        g.m, p->d_gen, sh, w.P, kd, st));
    else
      LAUNCH_OK(launch_raw_cols<float>(static_cast<float*>(cols) + p->col_off[g.first], g.count,
                                       g.m, p->d_gen, sh, w.P, kd, st));
  }
  return MTGP_OK;
}

int mtgp_fwht(void* x, int64_t batch, int32_t log2n, int32_t dtype, void* stream) {
  if (batch < 0 || log2n < 0 || log2n > 30) return MTGP_EINVAL;
  if (dtype != MTGP_DTYPE_F64 && dtype != MTGP_DTYPE_F32) return MTGP_EINVAL;
  if (batch == 0) return MTGP_OK;
  if (!x) return MTGP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = (int64_t)1 << log2n;
  const Sched sc;
  const size_t eb = dtype == MTGP_DTYPE_F64 ? sizeof(double) : sizeof(float);
  // Multi-pass sizes run in groups of at most 128 MiB of vectors, each group
  // through all its passes before the next: a group's working set then stays
  // in the 256 MB memory-side cache between passes (measured on [29][2^24]
  // FP64: 3.7 ms in groups against 5.1 ms for all vectors pass by pass).
  int64_t grp = batch;
  if (log2n > sc.a_bits) grp = std::max<int64_t>(1, ((int64_t)128 << 20) / (n * (int64_t)eb));
  for (int64_t b0 = 0; b0 < batch; b0 += grp) {
    const int64_t nb = std::min<int64_t>(grp, batch - b0);
    if (dtype == MTGP_DTYPE_F64)
      LAUNCH_OK(launch_fwht<double>(static_cast<double*>(x) + b0 * n, n, nb, log2n, sc, st));
    else
      LAUNCH_OK(launch_fwht<float>(static_cast<float*>(x) + b0 * n, n, nb, log2n, sc, st));
  }
  return MTGP_OK;
}

int mtgp_fft(const void* x, void* X, void* scratch, int64_t batch, int32_t log2n, int32_t dtype,
             int32_t bitrev_input, void* stream) {
  return fft_run(x, X, scratch, batch, log2n, dtype, bitrev_input, (hipStream_t)stream);
}

int mtgp_fft_noalloc(const void* x, void* X, int64_t batch, int32_t log2n, int32_t dtype,
                     int32_t bitrev_input, void* stream) {
  if (batch < 0 || batch > 65535 || log2n < 0 || log2n > 30) return MTGP_EINVAL;
  if (dtype != MTGP_DTYPE_F64 && dtype != MTGP_DTYPE_F32) return MTGP_EINVAL;
  if (batch == 0) return MTGP_OK;
  void* scr = nullptr;
  if (!lat_single_pass(log2n)) {
    const size_t cbytes = dtype == MTGP_DTYPE_F64 ? 2 * sizeof(double) : 2 * sizeof(float);
    // batch <= 65535 and log2n <= 30, so the product fits in 64 bits
    if ((uint64_t)batch * ((uint64_t)1 << log2n) * cbytes > (uint64_t)MTGP_FFT_NOALLOC_SCRATCH_BYTES)
      return MTGP_ETOOBIG;
    const int rc = fft_scratch_ptr(&scr);
    if (rc) return rc;
  }
  return fft_run(x, X, scr, batch, log2n, dtype, bitrev_input, (hipStream_t)stream);
}

int mtgp_set_data(const mtgp_plan* p, const double* y, void* ws, void* stream) {
  if (!p || !y || !ws) return MTGP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const WsView w = view(p, ws);
  // a fresh workspace reads as "no error" until the first evaluation
  LAUNCH_OK(launch_clear_status(w.status, st));
  if (p->family == MTGP_LAT) {
    // yhat_t = n_t^-1/2 F (bit reversal of y_t), in the spectrum layout of length n_t
    const KDesc kd = p->kd();
    const int nv = p->equal ? p->T : 1;
    for (int t = 0; t < p->T; t += nv) {
      LAUNCH_OK(launch_lat_forward<double, double>(
          LAT_SRC_Y, reinterpret_cast<cx<double>*>(w.pwork) + p->off[t],
          reinterpret_cast<cx<double>*>(w.yhat) + p->off[t], p->n[t], nv, p->m[t], y + p->off[t], 0,
          1.0 / std::sqrt((double)p->n[t]), nullptr, nullptr, nullptr, kd, st));
    }
  } else {
    HIP_OK(hipMemcpyAsync(w.yhat, y, (size_t)p->N * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int t = 0; t < p->T; t++) {
      LAUNCH_OK(launch_fwht<double>(w.yhat + p->off[t], p->n[t], 1, p->m[t], p->sched, st));
      LAUNCH_OK(launch_scale<double>(w.yhat + p->off[t], p->n[t],
                                     1.0 / std::sqrt((double)p->n[t]), st));
    }
  }
  if (solve_yh32(p))
    LAUNCH_OK(launch_narrow(w.yhat, w.yh32, p->N * (p->family == MTGP_LAT ? 2 : 1), st));
  return MTGP_OK;
}

int mtgp_nll(const mtgp_plan* p, const double* theta, double* out3, double* tau_hat, void* ws,
             void* stream) {
  if (!p || !theta || !out3 || !ws) return MTGP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
  return dispatch_loss(p, theta, out3, nullptr, tau_hat, ws, st, false);
}

int mtgp_nll_grad(const mtgp_plan* p, const double* theta, double* out3, double* grad,
                  double* tau_hat, void* ws, void* stream) {
  if (!p || !theta || !out3 || !grad || !ws) return MTGP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
  return dispatch_loss(p, theta, out3, grad, tau_hat, ws, st, false);
}

int mtgp_predict(const mtgp_plan* p, const double* theta, const uint32_t* xs, int64_t M,
                 double* mean, void* ws, void* stream) {
  if (!p || !theta || !ws || M < 0 || (M > 0 && (!xs || !mean))) return MTGP_EINVAL;
  if (M == 0) return MTGP_OK;
    hipStream_t st = (hipStream_t)stream;
  const WsView w = view(p, ws);
  int rc = dispatch_loss(p, theta, w.misc, nullptr, nullptr, ws, st, true);
  if (rc) return rc;
  double* alpha = w.ahat;
  if (p->family == MTGP_LAT) {
    // alpha (natural lattice order) = n^-1/2 F^H ahat = n^-1/2 Re F conj(ahat)
    const KDesc kd0 = p->kd();
    const int nv = p->equal ? p->T : 1;
    for (int t = 0; t < p->T; t += nv) {
      LAUNCH_OK(launch_lat_adjoint<double, double>(
          LAT_SINK_REAL, reinterpret_cast<const cx<double>*>(w.ahat) + p->off[t],
          reinterpret_cast<cx<double>*>(w.pwork) + p->off[t], w.alpha + p->off[t], p->n[t], nv,
          p->m[t], 1, 1.0 / std::sqrt((double)p->n[t]), p->d_gen, p->d_colshift, w.P, kd0, nullptr,
          st));
    }
    alpha = w.alpha;
  } else {
    // alpha_t = V_{m_t} ahat_t = H ahat_t / sqrt(n_t) (digital sequences: V real symmetric)
    for (int t = 0; t < p->T; t++) {
      LAUNCH_OK(launch_fwht<double>(w.ahat + p->off[t], p->n[t], 1, p->m[t], p->sched, st));
      LAUNCH_OK(launch_scale<double>(w.ahat + p->off[t], p->n[t], 1.0 / std::sqrt((double)p->n[t]), st));
    }
  }
  PredTasks pt;
  for (int t = 0; t < p->T; t++) {
    pt.m[t] = p->m[t];
    pt.off[t] = p->off[t];
  }
  const KDesc kd = p->kd();
  // chunking of the training points: about 2048 blocks in all, chunks of at
  // least 256 points; the spectrum buffer (free once alpha is formed) holds
  // the partial sums, test points are taken in batches that fit it
  const int64_t gx = (M + 255) / 256;
  const int64_t want = std::max<int64_t>(1, (2048 + gx - 1) / gx);
  PredChunks pc;
  pc.chunk = std::max<int64_t>(256, ((p->N + want - 1) / want + 255) / 256 * 256);
  pc.cstart[0] = 0;
  for (int t = 0; t < p->T; t++)
    pc.cstart[t + 1] = pc.cstart[t] + (int)((p->n[t] + pc.chunk - 1) / pc.chunk);
  // spectrum and working buffers (contiguous) are both free at this point
  const int64_t cap = (int64_t)((p->o_yhat - p->o_cols) / sizeof(double));
  const int64_t Mb = std::min<int64_t>(M, cap / pc.cstart[p->T]);
  if (Mb < 1) return MTGP_ENOMEM;
  double* part = reinterpret_cast<double*>(w.cols);
  for (int64_t m0 = 0; m0 < M; m0 += Mb) {
    const int64_t mb = std::min<int64_t>(Mb, M - m0);
    // the direct sum cancels heavily (alpha = Ktilde^-1 r is large where
    // Ktilde is ill conditioned), so it stays FP64 unless every column op is FP32
    if (p->precision != MTGP_F32)
      LAUNCH_OK(launch_predict_direct<double>(p->d_gen, p->d_taskshift, pt, pc, alpha,
                                              xs + (size_t)m0 * p->d, mb, w.P, kd, part,
                                              mean + (size_t)m0 * p->T, st));
    else
      LAUNCH_OK(launch_predict_direct<float>(p->d_gen, p->d_taskshift, pt, pc, alpha,
                                             xs + (size_t)m0 * p->d, mb, w.P, kd, part,
                                             mean + (size_t)m0 * p->T, st));
  }
  return MTGP_OK;
}

// scratch: T test-net columns of length max(n*, n_u) (FP64), T x n* folded
// spectra, the pair-shift table
static size_t prednet_layout(const mtgp_plan* p, int m_star, PredNet& pn, size_t& o_w,
                             size_t& o_sh) {
  // columns (complex for lattices), then the folded test spectra: nets
  // [T][n*]; lattices [T][n*] complex, the adjoint's working copy and the
  // real means [T][n*]
  const size_t cplx = p->family == MTGP_LAT ? 2 : 1;
  pn.T = p->T;
  pn.m_star = m_star;
  size_t o = 0;
  for (int u = 0; u < p->T; u++) {
    pn.m[u] = p->m[u];
    pn.col_off[u] = (int64_t)(o / sizeof(double));
    pn.task_off[u] = p->off[u];
    const int L = m_star > p->m[u] ? m_star : p->m[u];
    o += ((size_t)1 << L) * sizeof(double) * cplx;
  }
  o = align_up(o);
  o_w = o;
  o = align_up(o + ((size_t)1 << m_star) * p->T * sizeof(double) * (cplx == 2 ? 5 : 1));
  o_sh = o;
  o = align_up(o + (size_t)p->T * p->d * sizeof(uint32_t));
  return o;
}

size_t mtgp_predict_net_scratch_bytes(const mtgp_plan* p, int32_t m_star) {
  if (!p || m_star < 0 || m_star > 30) return 0;
  PredNet pn;
  size_t ow, osh;
  return prednet_layout(p, m_star, pn, ow, osh);
}

int mtgp_predict_net(const mtgp_plan* p, const double* theta, const uint32_t* shift_star,
                     int32_t m_star, double* mean, void* ws, void* scratch, void* stream) {
  if (!p || !theta || !shift_star || !mean || !ws || !scratch || m_star < 0 || m_star > 30)
    return MTGP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const WsView w = view(p, ws);
  // loss pass with ahat (and tau_used) at theta
  int rc = dispatch_loss(p, theta, w.misc, nullptr, nullptr, ws, st, true);
  if (rc) return rc;
  PredNet pn;
  size_t o_w, o_sh;
  prednet_layout(p, m_star, pn, o_w, o_sh);
  unsigned char* sb = static_cast<unsigned char*>(scratch);
  double* lam = reinterpret_cast<double*>(sb);
  double* wbuf = reinterpret_cast<double*>(sb + o_w);
  uint32_t* shd = reinterpret_cast<uint32_t*>(sb + o_sh);
  const bool lat = p->family == MTGP_LAT;
  std::vector<uint32_t> sh((size_t)p->T * p->d);
  for (int u = 0; u < p->T; u++)
    for (int j = 0; j < p->d; j++) {
      const uint32_t a = shift_star[j], b = p->shift[(size_t)u * p->d + j];
      sh[(size_t)u * p->d + j] = lat ? a - b : a ^ b;
    }
  LAUNCH_OK(launch_prednet_shifts(sh.data(), (int)sh.size(), shd, st));
  const KDesc kd = p->kd();
  if (lat) {
    const int64_t ns = (int64_t)1 << m_star;
    for (int u = 0; u < p->T; u++) {
      const int L = m_star > p->m[u] ? m_star : p->m[u];
      cx<double>* col = reinterpret_cast<cx<double>*>(lam + pn.col_off[u]);
      LAUNCH_OK(launch_lat_forward<double, double>(LAT_SRC_GEN, col, col, (int64_t)1 << L, 1, L,
                                                   nullptr, 0, 1.0, p->d_gen,
                                                   shd + (size_t)u * p->d, w.P, kd, st));
    }
    double* wwork = wbuf + 2 * ns * p->T;
    double* ureal = wwork + 2 * ns * p->T;
    LAUNCH_OK(launch_prednet_lat_fold(lam, pn, w.ahat, w.P, wbuf, st));
    LAUNCH_OK(launch_lat_adjoint<double, double>(
        LAT_SINK_REAL, reinterpret_cast<const cx<double>*>(wbuf),
        reinterpret_cast<cx<double>*>(wwork), ureal, ns, p->T, m_star, 1, 1.0, p->d_gen, shd, w.P,
        kd, nullptr, st));
    LAUNCH_OK(launch_prednet_lat_out(ureal, pn, w.P, mean, st));
    return MTGP_OK;
  }
  for (int u = 0; u < p->T; u++) {
    const int L = m_star > p->m[u] ? m_star : p->m[u];
    double* col = lam + pn.col_off[u];
    LAUNCH_OK(launch_gen_fwd<double, double>(col, (int64_t)1 << L, 1, L, p->d_gen,
                                             shd + (size_t)u * p->d, w.P, kd, p->sched, st));
    LAUNCH_OK(launch_strided<double, double, double>(col, col, col, (int64_t)1 << L, 1, L,
                                                     p->sched, st));
  }
  LAUNCH_OK(launch_prednet_fold(lam, pn, w.ahat, w.P, wbuf, st));
  LAUNCH_OK(launch_fwht<double>(wbuf, (int64_t)1 << m_star, p->T, m_star, p->sched, st));
  LAUNCH_OK(launch_prednet_out(wbuf, pn, w.P, mean, st));
  return MTGP_OK;
}

// scratch of mtgp_predict_var for batches of `batch` test points: the cross
// spectra (batch x N values, complex for lattices), their shifts, the
// partial quadratic forms and, at nested sizes, the batch x T stacked
// right-hand sides of the forward substitution
struct VarLayout {
  size_t o_shift, o_part, o_y, bytes;
  int nbx;
};
static VarLayout var_layout(const mtgp_plan* p, int64_t batch) {
  VarLayout L;
  const size_t cplx = p->family == MTGP_LAT ? 2 : 1;
  const int64_t nrow = p->equal ? p->n[0] : p->N;
  L.nbx = (int)std::min<int64_t>((nrow + 255) / 256, 256);
  size_t o = align_up((size_t)batch * p->N * sizeof(double) * cplx);
  L.o_shift = o;
  o = align_up(o + (size_t)p->T * batch * p->d * sizeof(uint32_t));
  L.o_part = o;
  o = align_up(o + (size_t)batch * L.nbx * std::max(16, p->T) * sizeof(double));
  L.o_y = o;
  if (!p->equal) o = align_up(o + (size_t)batch * p->T * p->N * sizeof(z2));
  L.bytes = o;
  return L;
}

size_t mtgp_predict_var_scratch_bytes(const mtgp_plan* p, int32_t batch) {
  if (!p || batch < 1) return 0;
  return var_layout(p, batch).bytes;
}

int mtgp_predict_var(const mtgp_plan* p, const double* theta, const uint32_t* xs, int64_t M,
                     int32_t batch, double* var, void* ws, void* scratch, void* stream) {
  if (!p || !theta || !ws || M < 0 || batch < 1 || (M > 0 && (!xs || !var || !scratch)))
    return MTGP_EINVAL;
  if (!p->equal && p->elim != MTGP_ELIM_SPARSE) return MTGP_ENOTSUP;
  if (M == 0) return MTGP_OK;
  hipStream_t st = (hipStream_t)stream;
  const WsView w = view(p, ws);
  // loss pass without gradient: the spectrum (equal sizes) or the factor in
  // the pattern storage (nested sizes) stays in ws
  int rc = dispatch_loss(p, theta, w.misc, nullptr, nullptr, ws, st, false);
  if (rc) return rc;
  const VarLayout L = var_layout(p, batch);
  unsigned char* sb = static_cast<unsigned char*>(scratch);
  double* mu = reinterpret_cast<double*>(sb);
  uint32_t* shd = reinterpret_cast<uint32_t*>(sb + L.o_shift);
  double* part = reinterpret_cast<double*>(sb + L.o_part);
  z2* Y = reinterpret_cast<z2*>(sb + L.o_y);
  const KDesc kd = p->kd();
  const bool lat = p->family == MTGP_LAT;
  for (int64_t m0 = 0; m0 < M; m0 += batch) {
    const int64_t mb = std::min<int64_t>(batch, M - m0);
    LAUNCH_OK(launch_var_shifts(xs + (size_t)m0 * p->d, mb, p->d_taskshift, p->T, p->d,
                                p->family, shd, st));
    // cross spectra of task u: mb columns of length n_u after mb * off[u]
    for (int u = 0; u < p->T; u++) {
      const int64_t len = p->n[u];
      const uint32_t* sh = shd + (size_t)u * mb * p->d;
      if (lat) {
        cx<double>* col = reinterpret_cast<cx<double>*>(mu) + (size_t)mb * p->off[u];
        LAUNCH_OK(launch_lat_forward<double, double>(LAT_SRC_GEN, col, col, len, (int)mb, p->m[u],
                                                     nullptr, 0, 1.0, p->d_gen, sh, w.P, kd, st));
      } else {
        double* col = mu + (size_t)mb * p->off[u];
        LAUNCH_OK(launch_gen_fwd<double, double>(col, len, (int)mb, p->m[u], p->d_gen, sh, w.P, kd,
                                                 p->sched, st));
        LAUNCH_OK(launch_strided<double, double, double>(col, col, col, len, mb, p->m[u],
                                                         p->sched, st));
      }
    }
    if (p->equal) {
      const int64_t n = p->n[0];
      if (p->precision == MTGP_FP64)
        LAUNCH_OK(launch_var_eq<double>(reinterpret_cast<const double*>(w.cols), n, p->pm,
                                        p->family, mu, mb, w.P, p->T, part, L.nbx, st));
      else
        LAUNCH_OK(launch_var_eq<float>(reinterpret_cast<const float*>(w.cols), n, p->pm,
                                       p->family, mu, mb, w.P, p->T, part, L.nbx, st));
      LAUNCH_OK(launch_var_finalize(part, L.nbx, mb, var_tm(p->T), true, w.P, kd,
                                    var + (size_t)m0 * p->T, st));
    } else {
      LAUNCH_OK(launch_var_nested(mu, p->a1, p->family, p->N, mb, w.P, w.a1a, Y, part, L.nbx, st));
      LAUNCH_OK(launch_var_finalize(part, L.nbx, mb, 0, false, w.P, kd, var + (size_t)m0 * p->T,
                                    st));
    }
  }
  return MTGP_OK;
}

int mtgp_gcv(const mtgp_plan* p, const double* theta, double* out3, double* grad,
             double* tau_hat, void* ws, void* stream) {
  if (!p || !theta || !out3 || !ws) return MTGP_EINVAL;
  if (!p->equal && p->elim != MTGP_ELIM_SPARSE) return MTGP_ENOTSUP;
  hipStream_t st = (hipStream_t)stream;
  if (!p->equal && grad) {
    switch (p->precision) {
      case MTGP_FP64: return run_gcv_nested_grad<double, double>(p, theta, out3, grad, tau_hat, ws, st);
      case MTGP_MIXED: return run_gcv_nested_grad<double, float>(p, theta, out3, grad, tau_hat, ws, st);
      default: return run_gcv_nested_grad<float, float>(p, theta, out3, grad, tau_hat, ws, st);
    }
  }
  if (!p->equal) {
    switch (p->precision) {
      case MTGP_FP64: return run_gcv_nested<double, double>(p, theta, out3, tau_hat, ws, st);
      case MTGP_MIXED: return run_gcv_nested<double, float>(p, theta, out3, tau_hat, ws, st);
      default: return run_gcv_nested<float, float>(p, theta, out3, tau_hat, ws, st);
    }
  }
  switch (p->precision) {
    case MTGP_FP64: return run_gcv<double, double>(p, theta, out3, grad, tau_hat, ws, st);
    case MTGP_MIXED: return run_gcv<double, float>(p, theta, out3, grad, tau_hat, ws, st);
    default: return run_gcv<float, float>(p, theta, out3, grad, tau_hat, ws, st);
  }
}

int mtgp_cubature(const mtgp_plan* p, const double* theta, double* mu_hat, double* Sigma,
                  void* ws, void* stream) {
  if (!p || !theta || !mu_hat || !Sigma || !ws) return MTGP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const WsView w = view(p, ws);
  // the loss leaves the spectrum (no gradient: it is not overwritten), ahat,
  // tau_used and, for nested sizes, Pi in the parameter block
  const int rc = dispatch_loss(p, theta, w.misc, nullptr, nullptr, ws, st, true);
  if (rc) return rc;
  CubDesc cd;
  cd.equal = p->equal ? 1 : 0;
  cd.n = p->n[0];
  for (int t = 0; t < MTGP_MAXT; t++)
    for (int u = 0; u < MTGP_MAXT; u++) cd.pair_col[t][u] = p->pm.col[t][u];
  for (int t = 0; t < p->T; t++) cd.task_off[t] = p->off[t];
  const KDesc kd = p->kd();
  if (p->precision == MTGP_FP64)
    LAUNCH_OK(launch_cubature<double>(reinterpret_cast<const double*>(w.cols), cd, w.ahat, w.P, kd,
                                      mu_hat, Sigma, st));
  else
    LAUNCH_OK(launch_cubature<float>(reinterpret_cast<const float*>(w.cols), cd, w.ahat, w.P, kd,
                                     mu_hat, Sigma, st));
  return MTGP_OK;
}

int mtgp_nll_grad_batched(int32_t nfits, mtgp_plan* const* plans, const double* const* thetas,
                          double* const* out3, double* const* grads, void* const* ws,
                          void* stream) {
  if (nfits < 0 || (nfits > 0 && (!plans || !thetas || !out3 || !grads || !ws))) return MTGP_EINVAL;
  for (int i = 0; i < nfits; i++) {
    const int rc = mtgp_nll_grad(plans[i], thetas[i], out3[i], grads[i], nullptr, ws[i], stream);
    if (rc) return rc;
  }
  return MTGP_OK;
}

// ---------------------------------------------------------------------------
// many fits, one launch per phase
// ---------------------------------------------------------------------------
}  // extern "C"

struct mtgp_batch {
  int nfits = 0;
  BFit* d_fits = nullptr;
  BItem* d_items = nullptr;  // column items grouped by (kernel type, width)
  struct Group {
    int kt, d, first, count;
  };
  std::vector<Group> groups;
  bool adam = false;
  int tmax = 0;  // largest T of the batch
};

namespace {

// per-fit slice of the batch workspace
struct BSlice {
  size_t o_S, o_logs, o_sp, o_ap, bytes;
};
BSlice batch_slice(const mtgp_plan* p) {
  BSlice b;
  size_t o = 0;
  b.o_S = o;
  o = align_up(o + (size_t)zf_elems(p->a1, p->N) * sizeof(z2));
  b.o_logs = o;
  o = align_up(o + (size_t)p->N * sizeof(double));
  b.o_sp = o;
  o = align_up(o + (size_t)BATCH_SOLVE_BLOCKS * solve_ns(p->T) * sizeof(double));
  b.o_ap = o;
  o = align_up(o + (size_t)p->ncol * adj_nq(p->d) * sizeof(double));
  b.bytes = o;
  return b;
}

int batch_check(int32_t nfits, mtgp_plan* const* plans) {
  if (nfits < 0 || (nfits > 0 && !plans)) return MTGP_EINVAL;
  for (int i = 0; i < nfits; i++) {
    const mtgp_plan* p = plans[i];
    if (!p) return MTGP_EINVAL;
    if (p->precision == MTGP_F32) return MTGP_ENOTSUP;
    if (p->m[0] > BATCH_MAX_M) return MTGP_ENOTSUP;
  }
  return MTGP_OK;
}

}  // namespace

extern "C" {

size_t mtgp_batch_workspace_bytes(int32_t nfits, mtgp_plan* const* plans) {
  if (batch_check(nfits, plans) != MTGP_OK) return 0;
  size_t total = 0;
  for (int i = 0; i < nfits; i++) total += batch_slice(plans[i]).bytes;
  return total;
}

int mtgp_batch_create(int32_t nfits, mtgp_plan* const* plans, void* const* ws,
                      double* const* thetas, double* const* out3, double* const* grads,
                      double* const* adam_m1, double* const* adam_m2, int64_t* const* adam_step,
                      const uint8_t* const* frozen, void* bws, mtgp_batch** out) {
  if (!out) return MTGP_EINVAL;
  *out = nullptr;
  int rc = batch_check(nfits, plans);
  if (rc) return rc;
  if (nfits > 0 && (!ws || !thetas || !out3 || !grads || !bws)) return MTGP_EINVAL;
  const bool adam = adam_m1 != nullptr;
  if (adam && (!adam_m2 || !adam_step)) return MTGP_EINVAL;
  std::vector<BFit> fits(nfits);
  struct Item {
    int kt, d, fit, col;
  };
  std::vector<Item> items;
  size_t bo = 0;
  for (int i = 0; i < nfits; i++) {
    const mtgp_plan* p = plans[i];
    if (!ws[i] || !thetas[i] || !out3[i] || !grads[i]) return MTGP_EINVAL;
    if (adam && (!adam_m1[i] || !adam_m2[i] || !adam_step[i])) return MTGP_EINVAL;
    const WsView w = view(p, ws[i]);
    const BSlice sl = batch_slice(p);
    unsigned char* b = static_cast<unsigned char*>(bws) + bo;
    bo += sl.bytes;
    BFit& F = fits[i];
    std::memset(&F, 0, sizeof(F));
    F.kd = p->kd();
    F.kd.unequal = 1;
    F.A = p->a1;
    F.ncol = p->ncol;
    F.sr_f32 = p->precision == MTGP_FP64 ? 0 : 1;
    F.N = p->N;
    F.gen = p->d_gen;
    F.colshift = p->d_colshift;
    F.colinfo = p->d_colinfo;
    F.theta = thetas[i];
    F.out3 = out3[i];
    F.grad = grads[i];
    F.P = w.P;
    F.status = w.status;
    F.cols = w.cols;
    F.work = reinterpret_cast<double*>(w.work);
    F.yhat = w.yhat;
    F.S = reinterpret_cast<z2*>(b + sl.o_S);
    F.logs = reinterpret_cast<double*>(b + sl.o_logs);
    F.sp = reinterpret_cast<double*>(b + sl.o_sp);
    F.ap = reinterpret_cast<double*>(b + sl.o_ap);
    if (adam) {
      F.m1 = adam_m1[i];
      F.m2 = adam_m2[i];
      F.step = adam_step[i];
      F.frozen = frozen ? frozen[i] : nullptr;
    }
    F.ntheta = theta_size(p);
    const int kt = kt_of(p->family, p->order, p->adaptive);
    for (int c = 0; c < p->ncol; c++) items.push_back({kt, p->d, i, c});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
    return a.kt != b.kt ? a.kt < b.kt : a.d < b.d;
  });
  mtgp_batch* bt = new (std::nothrow) mtgp_batch();
  if (!bt) return MTGP_ENOMEM;
  bt->nfits = nfits;
  bt->adam = adam;
  for (int i = 0; i < nfits; i++) bt->tmax = std::max(bt->tmax, plans[i]->T);
  // one launch per kernel type, at the widest dimension count of its fits
  // (narrower fits run with padding dimensions whose factor is exactly 1):
  // the column launches are bound by the latency of their largest columns,
  // so fewer, fuller launches beat exact widths
  std::vector<BItem> bi(items.size());
  for (size_t k = 0; k < items.size(); k++) {
    bi[k] = {items[k].fit, items[k].col};
    if (bt->groups.empty() || bt->groups.back().kt != items[k].kt)
      bt->groups.push_back({items[k].kt, items[k].d, (int)k, 0});
    bt->groups.back().d = std::max(bt->groups.back().d, items[k].d);
    bt->groups.back().count++;
  }
  if (nfits > 0) {
    if (hipMalloc(&bt->d_fits, fits.size() * sizeof(BFit)) != hipSuccess ||
        hipMalloc(&bt->d_items, bi.size() * sizeof(BItem)) != hipSuccess) {
      mtgp_batch_destroy(bt);
      return MTGP_ENOMEM;
    }
    if (hipMemcpy(bt->d_fits, fits.data(), fits.size() * sizeof(BFit), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(bt->d_items, bi.data(), bi.size() * sizeof(BItem), hipMemcpyHostToDevice) !=
            hipSuccess) {
      mtgp_batch_destroy(bt);
      return MTGP_EHIP;
    }
  }
  *out = bt;
  return MTGP_OK;
}

int mtgp_batch_destroy(mtgp_batch* b) {
  if (!b) return MTGP_OK;
  if (b->d_fits) (void)hipFree(b->d_fits);
  if (b->d_items) (void)hipFree(b->d_items);
  delete b;
  return MTGP_OK;
}

int mtgp_batch_nll_grad(const mtgp_batch* b, void* stream) {
  if (!b) return MTGP_EINVAL;
  if (b->nfits == 0) return MTGP_OK;
  hipStream_t st = (hipStream_t)stream;
  LAUNCH_OK(launch_batch_prep(b->d_fits, b->nfits, st));
  for (const auto& g : b->groups)
    LAUNCH_OK(launch_batch_fwd(b->d_fits, b->d_items + g.first, g.count, g.kt, g.d, st));
  LAUNCH_OK(launch_batch_solve(b->d_fits, b->nfits, b->tmax, st));
  for (const auto& g : b->groups)
    LAUNCH_OK(launch_batch_adj(b->d_fits, b->d_items + g.first, g.count, g.kt, g.d, st));
  LAUNCH_OK(launch_batch_final(b->d_fits, b->nfits, st));
  return MTGP_OK;
}

int mtgp_batch_adam_step(const mtgp_batch* b, double lr, double beta1, double beta2, double eps,
                         void* stream) {
  if (!b || !b->adam) return MTGP_EINVAL;
  LAUNCH_OK(launch_batch_adam(b->d_fits, b->nfits, lr, beta1, beta2, eps, (hipStream_t)stream));
  return MTGP_OK;
}

int mtgp_adam_step(double* theta, const double* grad, double* m1, double* m2, int64_t n, double lr,
                   double beta1, double beta2, double eps, int64_t* step, const uint8_t* frozen,
                   void* stream) {
  if (!theta || !grad || !m1 || !m2 || !step || n < 0 || n > 4096) return MTGP_EINVAL;
  LAUNCH_OK(launch_adam(theta, grad, m1, m2, n, lr, beta1, beta2, eps, step, frozen,
                        (hipStream_t)stream));
  return MTGP_OK;
}

int mtgp_status(const mtgp_plan* p, const void* ws, int64_t* bad_index) {
  if (!p || !ws) return MTGP_EINVAL;
  int st[4];
  const unsigned char* b = static_cast<const unsigned char*>(ws);
  if (hipMemcpy(st, b + p->o_status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return MTGP_EHIP;
  unsigned long long bad;
  std::memcpy(&bad, st + 2, sizeof(bad));
  if (bad_index) *bad_index = st[0] ? (int64_t)bad : -1;
  return st[0] ? MTGP_ENOTPD : MTGP_OK;
}

}  // extern "C"

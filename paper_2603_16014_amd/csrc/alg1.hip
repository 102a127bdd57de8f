// Nested unequal sample sizes: inverse and log-determinant of Lambda by
// block Gaussian elimination in task order (Algorithm "Inverse and
// log-determinant of Lambda"), with n_1 >= ... >= n_T.
//
// Structure (Theorem "Fast MTGP computations", item 3, tall case): for tasks
// t < u, Lambda_{(t,f),(u,g)} = sqrt(n_u / n_t) R_tu lambda_tu(f) when
// g = f mod n_u, else 0.  Hence rows couple only within residue classes, and
// after stage t (tasks 0..t bordered in) the running inverse A is block
// diagonal over residues r mod n_t with dense blocks of size
//   m_t = sum_{t' <= t} n_t' / n_t.
// Stage t merges, for each r mod n_t, the n_{t-1}/n_t blocks of residues
// r + k n_t (block diagonal, no coupling yet) and borders them with the one
// new row (t, r): with b the coupling column, L = A b, S = D - b^H L (a
// scalar: the Schur complement is diagonal), G = 1/S,
//   A <- [[A + L G L^H, -L G], [-G L^H, G]],   log det += log S.
// Rows of a stage-t block: the rows of child k = 0, 1, ... in order, then
// the new row.  Values are complex (lattices) or real with zero imaginary
// part (digital sequences); all arithmetic is FP64.
#include "kernels.h"

namespace mtgp {

__device__ inline z2 zm(z2 a, z2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline z2 zmc(z2 a, z2 b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }  // a conj(b)

// (task, frequency) of row q of the stage-s block with residue r
__device__ inline void decode_row(const Alg1Desc& A1, int s, int64_t r, int64_t q, int& task,
                                  int64_t& freq) {
  while (s > 0) {
    if (q == A1.msz[s] - 1) {
      task = s;
      freq = r;
      return;
    }
    const int64_t k = q / A1.msz[s - 1];
    q -= k * A1.msz[s - 1];
    r += k << A1.m[s];
    s--;
  }
  task = 0;
  freq = r;
}

// Coupling Lambda_{(t',g),(t,f)} for t' < t (g = f mod n_t by construction).
template <typename SR>
__device__ inline z2 coupling(const SR* cols, const Alg1Desc& A1, const Params* P, int family,
                              int tp, int64_t g, int t) {
  const z2 l = lam_at<SR>(cols, A1, family, A1.pc(tp, t), g);
  const double s = sqrt(ldexp(1.0, A1.m[t] - A1.m[tp])) * P->R[tp * MTGP_MAXT + t];
  return {s * l.x, s * l.y};
}

template <typename SR>
__device__ inline double diag_entry(const SR* cols, const Alg1Desc& A1, const Params* P, int family,
                                    int t, int64_t f) {
  return P->R[t * MTGP_MAXT + t] * lam_at<SR>(cols, A1, family, A1.pc(t, t), f).x + P->xi[t];
}

// Stage 0: A = 1 / Lambda_{(0,f),(0,f)} for each f < n_0.
template <typename SR>
__global__ void alg1_stage0_kernel(const SR* __restrict__ cols, Alg1Desc A1, const Params* P,
                                   int family, z2* __restrict__ Aout, double* __restrict__ logs,
                                   int* __restrict__ status) {
  const int64_t n0 = 1ll << A1.m[0];
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n0;
       f += (int64_t)gridDim.x * blockDim.x) {
    const double D = diag_entry<SR>(cols, A1, P, family, 0, f);
    if (!(D > 0.0) || !isfinite(D)) flag_bad(status, f);
    Aout[f] = {1.0 / D, 0.0};
    logs[f] = log(D);
  }
}

// Stage s >= 1: one block per residue r mod n_s.
template <typename SR>
__global__ __launch_bounds__(256) void alg1_stage_kernel(const SR* __restrict__ cols, Alg1Desc A1,
                                                         const Params* P, int family, int s,
                                                         const z2* __restrict__ Ain,
                                                         z2* __restrict__ Aout,
                                                         double* __restrict__ logs,
                                                         int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  const int64_t r = blockIdx.x;
  const int64_t mp = A1.msz[s - 1];          // child block size
  const int64_t K = 1ll << (A1.m[s - 1] - A1.m[s]);
  const int64_t ms = A1.msz[s];              // = K mp + 1
  const int64_t so = ms - 1;                 // old rows
  z2* b = reinterpret_cast<z2*>(smem);
  z2* L = b + so;
  // coupling of every old row to the new row (s, r)
  for (int64_t q = threadIdx.x; q < so; q += blockDim.x) {
    int tp;
    int64_t g;
    decode_row(A1, s, r, q, tp, g);
    b[q] = coupling<SR>(cols, A1, P, family, tp, g, s);
  }
  __syncthreads();
  // L = A_merged b, child by child
  for (int64_t q = threadIdx.x; q < so; q += blockDim.x) {
    const int64_t k = q / mp, ql = q - k * mp;
    const z2* Ak = Ain + (size_t)(r + (k << A1.m[s])) * mp * mp;
    z2 acc = {0.0, 0.0};
    for (int64_t c = 0; c < mp; c++) {
      const z2 p = zm(Ak[ql * mp + c], b[k * mp + c]);
      acc.x += p.x;
      acc.y += p.y;
    }
    L[q] = acc;
  }
  __syncthreads();
  double F = 0.0;
  for (int64_t q = threadIdx.x; q < so; q += blockDim.x) F += zmc(L[q], b[q]).x;  // Re(conj(b) L)
  F = block_sum(F, red);
  const double Sd = diag_entry<SR>(cols, A1, P, family, s, r) - F;
  if (threadIdx.x == 0) {
    if (!(Sd > 0.0) || !isfinite(Sd)) flag_bad(status, A1.stage_off[s] + r);
    logs[A1.stage_off[s] + r] = log(Sd);
  }
  const double G = 1.0 / Sd;
  z2* Ao = Aout + (size_t)r * ms * ms;
  for (int64_t e = threadIdx.x; e < ms * ms; e += blockDim.x) {
    const int64_t i = e / ms, j = e - i * ms;
    z2 v;
    if (i < so && j < so) {
      const z2 llh = zmc(L[i], L[j]);  // L_i conj(L_j)
      v = {llh.x * G, llh.y * G};
      const int64_t ki = i / mp, kj = j / mp;
      if (ki == kj) {
        const z2 a = Ain[(size_t)(r + (ki << A1.m[s])) * mp * mp + (i - ki * mp) * mp + (j - kj * mp)];
        v.x += a.x;
        v.y += a.y;
      }
    } else if (i < so) {
      v = {-L[i].x * G, -L[i].y * G};
    } else if (j < so) {
      v = {-L[j].x * G, L[j].y * G};  // -G conj(L_j)
    } else {
      v = {G, 0.0};
    }
    Ao[e] = v;
  }
}

// Profiled means from residue class 0: Pi_tu = sqrt(n_t n_u) (Lambda^-1)_{(t,0),(u,0)},
// (E K^-1 y)_t = sqrt(n_t) (Lambda^-1 yhat)_{(t,0)}; Pi tau = E K^-1 y (Theorem
// "Fast MTGP computations", item 4).  Writes P->Pi and P->tau_used.  One block.
__global__ void alg1_tau_kernel(Alg1Desc A1, Params* P, const double* __restrict__ yhat,
                                int family, int profile, const z2* __restrict__ Afin) {
  __shared__ double Pi[MTGP_MAXT][MTGP_MAXT + 1];
  __shared__ int64_t rowof[MTGP_MAXT];
  const int T = A1.T;
  const int s = T - 1;
  const int64_t ms = A1.msz[s];
  if (threadIdx.x == 0) {
    for (int64_t q = 0; q < ms; q++) {
      int t;
      int64_t f;
      decode_row(A1, s, 0, q, t, f);
      if (f == 0) rowof[t] = q;
    }
  }
  __syncthreads();
  // rows (t, 0) of the residue-0 block of Lambda^-1
  for (int e = threadIdx.x; e < T * (T + 1); e += blockDim.x) {
    const int t = e / (T + 1), u = e - t * (T + 1);
    const int64_t qt = rowof[t];
    if (u < T) {
      Pi[t][u] = sqrt(ldexp(1.0, A1.m[t] + A1.m[u])) * Afin[qt * ms + rowof[u]].x;
    } else {
      double acc = 0.0;
      for (int64_t c = 0; c < ms; c++) {
        int tc;
        int64_t fc;
        decode_row(A1, s, 0, c, tc, fc);
        const int64_t yp = A1.task_off[tc] + spec_pos(family, fc, A1.m[tc]);
        const double yr = family == FAM_DSEQ ? yhat[yp] : yhat[2 * yp];
        const double yi = family == FAM_DSEQ ? 0.0 : yhat[2 * yp + 1];
        const z2 a = Afin[qt * ms + c];
        acc += a.x * yr - a.y * yi;
      }
      Pi[t][T] = sqrt(ldexp(1.0, A1.m[t])) * acc;
    }
  }
  __syncthreads();
  // Pi itself (Bayesian cubature reads it)
  for (int e = threadIdx.x; e < T * T; e += blockDim.x)
    P->Pi[(e / T) * MTGP_MAXT + e % T] = Pi[e / T][e % T];
  if (!profile) {
    if (threadIdx.x < T) P->tau_used[threadIdx.x] = P->tau[threadIdx.x];
    return;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < T; c++) {  // Gaussian elimination with partial pivoting
      int pv = c;
      for (int i = c + 1; i < T; i++)
        if (fabs(Pi[i][c]) > fabs(Pi[pv][c])) pv = i;
      for (int k = 0; k <= T; k++) {
        const double tmp = Pi[c][k];
        Pi[c][k] = Pi[pv][k];
        Pi[pv][k] = tmp;
      }
      for (int i = c + 1; i < T; i++) {
        const double fct = Pi[i][c] / Pi[c][c];
        for (int k = c; k <= T; k++) Pi[i][k] -= fct * Pi[c][k];
      }
    }
    double tau[MTGP_MAXT];
    for (int c = T - 1; c >= 0; c--) {
      double acc = Pi[c][T];
      for (int k = c + 1; k < T; k++) acc -= Pi[c][k] * tau[k];
      tau[c] = acc / Pi[c][c];
    }
    for (int t = 0; t < T; t++) P->tau_used[t] = tau[t];
  }
}

// Final residue classes r mod n_T: ahat = Lambda^-1 rhat, quad, and for the
// gradient W = Lambda^-1 - ahat ahat^H on Lambda's pattern:
//   omega_tu(f) = 2 sqrt(n_u/n_t) conj(W_{(t,f),(u,f mod n_u)})  (t < u; R_tu
//   is applied to the pair column's sums in the chain rule),
//   omega_diag col(f) += R_tt W_{(t,f),(t,f)},  G_tt, sum_f W_tt, ahat(0).
// Partials per block use the solve layout (solve_ns) with TM = solve_tm(T).
template <typename SR, int TM>
__global__ __launch_bounds__(256) void alg1_final_kernel(SR* __restrict__ cols, Alg1Desc A1,
                                                         const Params* P, int family, int grad,
                                                         const double* __restrict__ yhat,
                                                         const z2* __restrict__ Afin,
                                                         double* __restrict__ ahat,
                                                         double* __restrict__ partials) {
  constexpr int NQ = 2 + 3 * TM;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[4 * NQ];
  const int T = A1.T, s = T - 1;
  const int64_t r = blockIdx.x;
  const int64_t ms = A1.msz[s];
  z2* rh = reinterpret_cast<z2*>(smem);  // rhat, then ahat
  z2* ah = rh + ms;
  int* tsk = reinterpret_cast<int*>(ah + ms);
  int64_t* frq = reinterpret_cast<int64_t*>(tsk + ((ms + 1) & ~1ll));
  for (int64_t q = threadIdx.x; q < ms; q += blockDim.x) {
    int t;
    int64_t f;
    decode_row(A1, s, r, q, t, f);
    tsk[q] = t;
    frq[q] = f;
    const int64_t yp = A1.task_off[t] + spec_pos(family, f, A1.m[t]);
    z2 y = family == FAM_DSEQ ? z2{yhat[yp], 0.0} : z2{yhat[2 * yp], yhat[2 * yp + 1]};
    if (f == 0) y.x -= sqrt(ldexp(1.0, A1.m[t])) * P->tau_used[t];
    rh[q] = y;
  }
  __syncthreads();
  const z2* A = Afin + (size_t)r * ms * ms;
  double vals[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) vals[q] = 0.0;
  for (int64_t q = threadIdx.x; q < ms; q += blockDim.x) {
    z2 acc = {0.0, 0.0};
    for (int64_t c = 0; c < ms; c++) {
      const z2 p = zm(A[q * ms + c], rh[c]);
      acc.x += p.x;
      acc.y += p.y;
    }
    ah[q] = acc;
    vals[0] += zmc(acc, rh[q]).x;  // Re(conj(rhat) ahat)
  }
  __syncthreads();
  for (int64_t q = threadIdx.x; q < ms; q += blockDim.x) {
    const int t = tsk[q];
    const int64_t f = frq[q];
    if (ahat) {
      const int64_t yp = A1.task_off[t] + spec_pos(family, f, A1.m[t]);
      if (family == FAM_DSEQ) {
        ahat[yp] = ah[q].x;
      } else {
        ahat[2 * yp] = ah[q].x;
        ahat[2 * yp + 1] = ah[q].y;
      }
    }
    if (f == 0) {
#pragma unroll
      for (int i = 0; i < TM; i++)
        if (i == t) vals[2 + 2 * TM + i] = ah[q].x;
    }
  }
  if (grad) {
    // diagonal entries: one diagonal column per distinct length; the rows of
    // equal-length tasks at one frequency all live in this block, each
    // diagonal-column position is written by the thread owning the row of
    // the first task with that length
    for (int64_t q = threadIdx.x; q < ms; q += blockDim.x) {
      const int t = tsk[q];
      const int64_t f = frq[q];
      const z2 aq = ah[q];
      const double w = A[q * ms + q].x - (aq.x * aq.x + aq.y * aq.y);
      const double lam = lam_at<SR>(cols, A1, family, A1.pc(t, t), f).x;
#pragma unroll
      for (int i = 0; i < TM; i++) {
        if (i == t) {
          vals[2 + i] += w * lam;
          vals[2 + TM + i] += w;
        }
      }
    }
    // every read of the diagonal columns above precedes the writes below
    // (tasks of equal length share one diagonal column)
    __syncthreads();
    for (int64_t q = threadIdx.x; q < ms; q += blockDim.x) {
      const int t = tsk[q];
      const int64_t f = frq[q];
      const z2 aq = ah[q];
      if (A1.df(t) == t) {
        double wsum = 0.0;
        // rows of the other tasks with the same length and the same frequency
        for (int64_t q2 = 0; q2 < ms; q2++) {
          const int t2 = tsk[q2];
          if (A1.m[t2] == A1.m[t] && frq[q2] == f) {
            const z2 a2 = ah[q2];
            wsum += P->R[t2 * MTGP_MAXT + t2] * (A[q2 * ms + q2].x - (a2.x * a2.x + a2.y * a2.y));
          }
        }
        const int c = A1.pc(t, t);
        const int64_t pos = A1.col_off[c] + spec_pos(family, f, A1.m[t]);
        if (family == FAM_DSEQ) {
          cols[pos] = (SR)wsum;
        } else {
          cols[2 * pos] = (SR)wsum;
          cols[2 * pos + 1] = (SR)0;
        }
      }
      // off-diagonal pattern entries: partner rows (u, f mod n_u), u > t
      for (int u = t + 1; u < T; u++) {
        const int64_t g = f & ((1ll << A1.m[u]) - 1);
        // locate the partner row: scan (block rows are few per task)
        int64_t qu = -1;
        for (int64_t q2 = 0; q2 < ms; q2++)
          if (tsk[q2] == u && frq[q2] == g) {
            qu = q2;
            break;
          }
        if (qu < 0) continue;  // cannot happen: g = f mod n_u lies in this residue class
        const z2 au = ah[qu];
        const z2 Atu = A[q * ms + qu];
        const z2 aa = zmc(aq, au);  // a_t conj(a_u)
        const z2 wtu = {Atu.x - aa.x, Atu.y - aa.y};
        const double sc = sqrt(ldexp(1.0, A1.m[u] - A1.m[t]));
        const double R2 = 2.0 * sc;
        const int c = A1.pc(t, u);
        const int64_t pos = A1.col_off[c] + spec_pos(family, f, A1.m[t]);
        if (family == FAM_DSEQ) {
          cols[pos] = (SR)(R2 * wtu.x);
        } else {
          cols[2 * pos] = (SR)(R2 * wtu.x);
          cols[2 * pos + 1] = (SR)(-R2 * wtu.y);
        }
      }
    }
  }
  block_sum_store<NQ>(vals, NQ, red, partials + (size_t)blockIdx.x * NQ);
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
template <typename SR>
int launch_alg1(SR* cols, const Alg1Desc& A1, Params* P, int family, bool grad,
                const double* yhat, z2* bufA, z2* bufB, double* logs, double* ahat,
                double* partials, int* status, hipStream_t st) {
  const int T = A1.T;
  z2* cur = bufA;
  z2* nxt = bufB;
  {
    const int64_t n0 = 1ll << A1.m[0];
    int64_t blocks = (n0 + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(alg1_stage0_kernel<SR>, dim3((unsigned)blocks), dim3(256), 0, st, cols, A1,
                       P, family, cur, logs, status);
  }
  for (int s = 1; s < T; s++) {
    const size_t lds = (size_t)(A1.msz[s] - 1) * 2 * sizeof(z2);
    hipLaunchKernelGGL(alg1_stage_kernel<SR>, dim3((unsigned)(1u << A1.m[s])), dim3(256), lds, st,
                       cols, A1, P, family, s, cur, nxt, logs, status);
    z2* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  hipLaunchKernelGGL(alg1_tau_kernel, dim3(1), dim3(256), 0, st, A1, P, yhat, family,
                     A1.profile, cur);
  const int64_t ms = A1.msz[T - 1];
  const size_t lds = (size_t)ms * 2 * sizeof(z2) + ((ms + 1) & ~1ll) * sizeof(int) +
                     (size_t)ms * sizeof(int64_t);
  const dim3 grid((unsigned)(1u << A1.m[T - 1]));
#define MTGP_FIN(TMV)                                                                          \
  hipLaunchKernelGGL((alg1_final_kernel<SR, TMV>), grid, dim3(256), lds, st, cols, A1, P,      \
                     family, grad ? 1 : 0, yhat, cur, ahat, partials)
  if (T <= 1) MTGP_FIN(1);
  else if (T <= 2) MTGP_FIN(2);
  else if (T <= 4) MTGP_FIN(4);
  else if (T <= 8) MTGP_FIN(8);
  else MTGP_FIN(16);
#undef MTGP_FIN
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_alg1<double>(double*, const Alg1Desc&, Params*, int, bool, const double*, z2*,
                                 z2*, double*, double*, double*, int*, hipStream_t);
template int launch_alg1<float>(float*, const Alg1Desc&, Params*, int, bool, const double*, z2*,
                                z2*, double*, double*, double*, int*, hipStream_t);

}  // namespace mtgp

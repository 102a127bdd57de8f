// Device bodies of the fill-free task-order elimination (see elim.hip for
// the method), written over an index range [start, total) with a stride so
// that the same code runs as grid-wide kernels (elim.hip, one launch per
// stage) and inside one workgroup per fit (batch.hip, stages separated by
// barriers).
#pragma once
#include "kernels.h"

namespace mtgp {


namespace {

__device__ inline z2 zmul(z2 a, z2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline z2 zmulc(z2 a, z2 b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
__device__ inline z2 zconj(z2 a) { return {a.x, -a.y}; }
__device__ inline z2 zsub(z2 a, z2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline z2 zscale(z2 a, double s) { return {a.x * s, a.y * s}; }

// pattern entry of row (b, g mod n_b), column (a, g), a <= b
__device__ inline int64_t pidx(const Alg1Desc& A, int a, int b, int64_t g) {
  return A.so[a] + ((int64_t)(b - a) << A.m[a]) + g;
}

// task of a flat index given increasing offsets off[0..T)
__device__ inline int task_of(const int64_t* off, int T, int64_t i) {
  int t = 0;
  while (t + 1 < T && i >= off[t + 1]) t++;
  return t;
}


}  // namespace

// complex load / store through generic or global-qualified pointers
template <typename P>
__device__ inline z2 zld(P p, int64_t i) {
  return {p[i].x, p[i].y};
}
template <typename P>
__device__ inline void zst(P p, int64_t i, z2 v) {
  p[i].x = v.x;
  p[i].y = v.y;
}

// Pattern values from the spectrum, yhat in natural frequency order, unit
// right-hand sides.  Grid-stride over so[T] + N + T ms entries.
// (CP, PP, YP, ZP: pointer types, generic or global-qualified.)
template <typename SR, typename CP, typename PP, typename YP, typename ZP>
__device__ inline void zf_init_body(CP cols, const Alg1Desc& A, PP P, int family, int64_t N,
                                    YP yhat, ZP S, ZP rr, ZP U, int64_t start, int64_t stride) {
  const int T = A.T;
  const int64_t nS = A.so[T], ms = A.msz[T - 1];
  const int64_t total = nS + N + (int64_t)T * ms;
  for (int64_t i = start; i < total; i += stride) {
    if (i < nS) {
      const int a = task_of(A.so, T, i);
      const int64_t r = i - A.so[a];
      const int b = a + (int)(r >> A.m[a]);
      const int64_t g = r & ((1ll << A.m[a]) - 1);
      const int c = A.pc(a, b);
      const int64_t lp = A.col_off[c] + spec_pos(family, g, A.col_m[c]);
      const z2 l = family == FAM_DSEQ ? z2{(double)cols[lp], 0.0}
                                      : z2{(double)cols[2 * lp], (double)cols[2 * lp + 1]};
      if (b == a) {
        zst(S, i, z2{P->R[a * MTGP_MAXT + a] * l.x + P->xi[a], 0.0});
      } else {
        // Lambda_{(a,g),(b,g mod n_b)} = sqrt(n_b / n_a) R_ab lambda_ab(g); the
        // stored entry (row (b, .), column (a, g)) is its conjugate
        const double sc = sqrt(ldexp(1.0, A.m[b] - A.m[a])) * P->R[a * MTGP_MAXT + b];
        zst(S, i, zconj(zscale(l, sc)));
      }
    } else if (i < nS + N) {
      const int64_t q = i - nS;
      const int t = task_of(A.task_off, T, q);
      const int64_t f = q - A.task_off[t];
      const int64_t yp = A.task_off[t] + spec_pos(family, f, A.m[t]);
      zst(rr, q, family == FAM_DSEQ ? z2{yhat[yp], 0.0} : z2{yhat[2 * yp], yhat[2 * yp + 1]});
    } else {
      const int64_t q = i - nS - N;
      const int64_t v = q / ms, node = q - v * ms;
      zst(U, q, z2{node == A.coff[v] ? 1.0 : 0.0, 0.0});
    }
  }
}

// Stage t, later task u: the n_u (T - u) pattern targets S_uv[g], the n_u
// targets rr(u, g) and the T (n_u / n_T) unit targets of class 0.  Each
// target sums n_t / n_u terms; a group of G lanes (power of two <= 64) of
// one wave shares a target.
// (ZP: pointer type, generic or global-qualified.)
template <typename ZP>
__device__ inline void zf_factor_body(const Alg1Desc& A, int t, int u, int G, ZP S, ZP rr, ZP U,
                                      int64_t start, int64_t stride) {
  const int T = A.T;
  const int64_t nu = 1ll << A.m[u];
  const int64_t K = 1ll << (A.m[t] - A.m[u]);  // terms per target
  const int cs = A.m[T - 1];
  const int64_t cu = nu >> cs;                 // class-0 nodes of task u
  const int64_t ms = A.msz[T - 1];
  const int64_t ntarget = (int64_t)(T - u) * nu + nu + (int64_t)T * cu;
  const int lane = threadIdx.x & (G - 1);
  const int64_t gstride = stride / G;
  for (int64_t q = start / G;
       q < ((ntarget + gstride - 1) / gstride) * gstride; q += gstride) {
    // every lane of a group runs the same number of iterations (shuffles)
    const bool live = q < ntarget;
    z2 acc = {0.0, 0.0};
    int kind = 0;
    int64_t g = 0, dst = 0;
    int v = u, rv = 0;
    if (live) {
      if (q < (int64_t)(T - u) * nu) {
        v = u + (int)(q >> A.m[u]);
        g = q & (nu - 1);
        dst = pidx(A, u, v, g);
        for (int64_t j = lane; j < K; j += G) {
          const int64_t f = g + (j << A.m[u]);
          const double d = zld(S, pidx(A, t, t, f)).x;
          const z2 p = zmulc(zld(S, pidx(A, t, v, f)), zld(S, pidx(A, t, u, f)));
          acc.x += p.x / d;
          acc.y += p.y / d;
        }
      } else if (q < (int64_t)(T - u) * nu + nu) {
        kind = 1;
        g = q - (int64_t)(T - u) * nu;
        dst = A.task_off[u] + g;
        for (int64_t j = lane; j < K; j += G) {
          const int64_t f = g + (j << A.m[u]);
          const double d = zld(S, pidx(A, t, t, f)).x;
          const z2 p = zmul(zld(S, pidx(A, t, u, f)), zld(rr, A.task_off[t] + f));
          acc.x += p.x / d;
          acc.y += p.y / d;
        }
      } else {
        kind = 2;
        const int64_t r = q - (int64_t)(T - u) * nu - nu;
        rv = (int)(r / cu);
        const int64_t k = r - (int64_t)rv * cu;
        g = k << cs;
        dst = (int64_t)rv * ms + A.coff[u] + k;
        for (int64_t j = lane; j < K; j += G) {
          const int64_t f = g + (j << A.m[u]);
          const double d = zld(S, pidx(A, t, t, f)).x;
          const z2 p = zmul(zld(S, pidx(A, t, u, f)), zld(U, (int64_t)rv * ms + A.coff[t] + (f >> cs)));
          acc.x += p.x / d;
          acc.y += p.y / d;
        }
      }
    }
    for (int o = G >> 1; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, 64);
      acc.y += __shfl_xor(acc.y, o, 64);
    }
    if (live && lane == 0) {
      if (kind == 0) {
        const z2 s = zld(S, dst);
        zst(S, dst, v == u ? z2{s.x - acc.x, 0.0} : zsub(s, acc));
      } else if (kind == 1) {
        zst(rr, dst, zsub(zld(rr, dst), acc));
      } else {
        zst(U, dst, zsub(zld(U, dst), acc));
      }
    }
  }
}

// S position of the Lambda^-1 entry between (u, g_u) and (v, g_v), u, v > t,
// in the overwritten (inverse) pattern storage; zpair_val turns the stored
// value into the entry (diagonal: its real part; u < v: the conjugate).
__device__ inline int64_t zpair_idx(const Alg1Desc& A, int u, int v, int64_t gu, int64_t gv) {
  return u <= v ? pidx(A, u, v, gu) : pidx(A, v, u, gv);
}
__device__ inline z2 zpair_val(z2 s, int u, int v) {
  if (u == v) return {s.x, 0.0};
  return u < v ? zconj(s) : s;
}

// Backward stage t over the nodes (t, f): pivot check and log, ahat of the
// data (and, on residue class 0, of the unit right-hand sides); with GRAD
// the inverse entries of the column of (t, f), written over it.
//
// Every load of a group is issued before its first use, with no branch in
// between: slots of tasks outside (t, T) read a valid entry (the node's own
// diagonal or right-hand side) and are skipped in the arithmetic, which
// runs in the same order as with the slots skipped outright.  (Loads behind
// branches of their own are waited for one by one.)  ZP, DP and IP are the
// pointer types (generic, or global for pointers read from memory).
template <int TM, bool GRAD, typename ZP, typename DP, typename IP>
__device__ inline void zf_back_body(const Alg1Desc& A, int t, ZP S, ZP rr, ZP U, DP logs,
                                    IP status, int64_t start, int64_t stride) {
  const int T = A.T;
  const int64_t nt = 1ll << A.m[t];
  const int cs = A.m[T - 1];
  const int64_t ms = A.msz[T - 1];
  for (int64_t f = start; f < nt; f += stride) {
    const int64_t node = A.task_off[t] + f;
    const int64_t dix = pidx(A, t, t, f);
    const double d = zld(S, dix).x;
    z2 Lr[TM], rv[TM];
#pragma unroll
    for (int u = 0; u < TM; u++) {
      const bool act = u > t && u < T;
      Lr[u] = zld(S, act ? pidx(A, t, u, f) : dix);
      rv[u] = zld(rr, act ? A.task_off[u] + (f & ((1ll << A.m[u]) - 1)) : node);
    }
    const z2 rn = zld(rr, node);
    if (!(d > 0.0) || !isfinite(d)) flag_bad((int*)status, node);
    logs[node] = log(d);
    const double di = 1.0 / d;
    z2 L[TM];
#pragma unroll
    for (int u = 0; u < TM; u++) L[u] = (u > t && u < T) ? zscale(Lr[u], di) : z2{0.0, 0.0};
    // ahat(t, f) = z / d - sum_u conj(L_u) ahat(u, f mod n_u)
    z2 a = zscale(rn, di);
#pragma unroll
    for (int u = 0; u < TM; u++)
      if (u > t && u < T) a = zsub(a, zmulc(rv[u], L[u]));  // conj(L_u) x = x conj(L_u)
    zst(rr, node, a);
    if ((f & ((1ll << cs) - 1)) == 0) {
      const int64_t k = f >> cs;
      for (int v = 0; v < T; v++) {
        ZP Uv = U + (int64_t)v * ms;
        z2 b = zscale(zld(Uv, A.coff[t] + k), di);
#pragma unroll
        for (int u = 0; u < TM; u++)
          if (u > t && u < T)
            b = zsub(b, zmulc(zld(Uv, A.coff[u] + ((f & ((1ll << A.m[u]) - 1)) >> cs)), L[u]));
        zst(Uv, A.coff[t] + k, b);
      }
    }
    if constexpr (GRAD) {
      z2 Zc[TM];
      double ztt = di;
#pragma unroll
      for (int u = 0; u < TM; u++) {
        Zc[u] = {0.0, 0.0};
        if (u > t && u < T) {
          const int64_t gu = f & ((1ll << A.m[u]) - 1);
          z2 zs[TM];
#pragma unroll
          for (int v = 0; v < TM; v++) {
            const bool act = v > t && v < T;
            zs[v] = zld(S, act ? zpair_idx(A, u, v, gu, f & ((1ll << A.m[v]) - 1)) : dix);
          }
          z2 acc = {0.0, 0.0};
#pragma unroll
          for (int v = 0; v < TM; v++)
            if (v > t && v < T) {
              const z2 p = zmul(zpair_val(zs[v], u, v), L[v]);
              acc.x += p.x;
              acc.y += p.y;
            }
          Zc[u] = {-acc.x, -acc.y};
          ztt -= zmulc(L[u], Zc[u]).x;  // Re(conj(Z_u) L_u)
        }
      }
      zst(S, dix, z2{ztt, 0.0});
#pragma unroll
      for (int u = 0; u < TM; u++)
        if (u > t && u < T) zst(S, pidx(A, t, u, f), Zc[u]);
    }
  }
}

// Profiled means from residue class 0 (one block): Pi_tu = sqrt(n_t n_u)
// (Lambda^-1)_{(t,0),(u,0)}, (E K^-1 y)_t = sqrt(n_t) (Lambda^-1 yhat)_{(t,0)};
// Pi tau = E K^-1 y.  Writes P->Pi and P->tau_used.
__device__ inline void zf_tau_body(const Alg1Desc& A, Params* P, const z2* __restrict__ rr,
                              const z2* __restrict__ U) {
  __shared__ double Pi[MTGP_MAXT][MTGP_MAXT + 1];
  const int T = A.T;
  const int64_t ms = A.msz[T - 1];
  for (int e = threadIdx.x; e < T * (T + 1); e += blockDim.x) {
    const int t = e / (T + 1), u = e - t * (T + 1);
    if (u < T)
      Pi[t][u] = sqrt(ldexp(1.0, A.m[t] + A.m[u])) * U[(int64_t)u * ms + A.coff[t]].x;
    else
      Pi[t][T] = sqrt(ldexp(1.0, A.m[t])) * rr[A.task_off[t]].x;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < T * T; e += blockDim.x)
    P->Pi[(e / T) * MTGP_MAXT + e % T] = Pi[e / T][e % T];
  if (!A.profile) {
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
    for (int c = 0; c < T; c++) P->tau_used[c] = tau[c];
  }
}

namespace {
// ahat of node (u, g) for the means used: Lambda^-1 yhat minus the unit
// solutions on residue class 0
__device__ inline z2 ahat_at(const Alg1Desc& A, const Params* P, const z2* rr, const z2* U, int u,
                             int64_t g) {
  z2 a = rr[A.task_off[u] + g];
  const int cs = A.m[A.T - 1];
  if ((g & ((1ll << cs) - 1)) == 0) {
    const int64_t ms = A.msz[A.T - 1];
    const int64_t k = A.coff[u] + (g >> cs);
    for (int v = 0; v < A.T; v++) {
      const double c = sqrt(ldexp(1.0, A.m[v])) * P->tau_used[v];
      const z2 e = U[(int64_t)v * ms + k];
      a.x -= c * e.x;
      a.y -= c * e.y;
    }
  }
  return a;
}
}  // namespace

// ahat_at through generic or global-qualified pointers
template <typename PP, typename ZP>
__device__ inline z2 ahat_at_p(const Alg1Desc& A, PP P, ZP rr, ZP U, int u, int64_t g) {
  z2 a = zld(rr, A.task_off[u] + g);
  const int cs = A.m[A.T - 1];
  if ((g & ((1ll << cs) - 1)) == 0) {
    const int64_t ms = A.msz[A.T - 1];
    const int64_t k = A.coff[u] + (g >> cs);
    for (int v = 0; v < A.T; v++) {
      const double c = sqrt(ldexp(1.0, A.m[v])) * P->tau_used[v];
      const z2 e = zld(U, (int64_t)v * ms + k);
      a.x -= c * e.x;
      a.y -= c * e.y;
    }
  }
  return a;
}

// Final pass over all nodes: quad = Re(rhat^H ahat), ahat out, a0; with the
// gradient W = Lambda^-1 - ahat ahat^H on the pattern, written as adjoint
// weights over the spectrum (the layout of the unequal-size elimination):
//   pair column (t, u), t < u, at f: 2 sqrt(n_u / n_t) conj(W_{(t,f),(u,f mod n_u)});
//   diagonal column of length n_t at f: sum over tasks t2 of that length of
//   R_{t2 t2} W_{(t2,f),(t2,f)}, formed (with G_tt and sum W_tt) by the
//   node of the first such task, which alone reads and writes that entry.
// CP, PP, YP and ZP are the pointer types (generic, or global for pointers
// read from memory).
template <typename SR, int TM, typename CP, typename PP, typename YP, typename ZP>
__device__ inline void zf_final_body(CP cols, const Alg1Desc& A, int64_t N, PP P, int family,
                                     int grad, YP yhat, ZP S, ZP rr, ZP U,
                                     double* __restrict__ ahat, double* __restrict__ row,
                                     int64_t start, int64_t stride) {
  constexpr int NQ = 2 + 3 * TM;
  __shared__ double red[4 * NQ];
  const int T = A.T;
  double vals[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) vals[q] = 0.0;
  for (int64_t node = start; node < N; node += stride) {
    const int t = task_of(A.task_off, T, node);
    const int64_t f = node - A.task_off[t];
    const int64_t yp = A.task_off[t] + spec_pos(family, f, A.m[t]);
    z2 y = family == FAM_DSEQ ? z2{yhat[yp], 0.0} : z2{yhat[2 * yp], yhat[2 * yp + 1]};
    if (f == 0) y.x -= sqrt(ldexp(1.0, A.m[t])) * P->tau_used[t];
    const z2 a = ahat_at_p(A, P, rr, U, t, f);
    vals[0] += zmulc(a, y).x;  // Re(conj(rhat) ahat)
    if (ahat) {
      if (family == FAM_DSEQ) {
        ahat[yp] = a.x;
      } else {
        ahat[2 * yp] = a.x;
        ahat[2 * yp + 1] = a.y;
      }
    }
    if (f == 0) {
#pragma unroll
      for (int i = 0; i < TM; i++)
        if (i == t) vals[2 + 2 * TM + i] = a.x;
    }
    if (!grad) continue;
    if (A.df(t) == t) {
      const int c = A.pc(t, t);
      const int64_t lp = A.col_off[c] + spec_pos(family, f, A.col_m[c]);
      const double lam = (double)cols[family == FAM_DSEQ ? lp : 2 * lp];
      double wsum = 0.0;
#pragma unroll
      for (int i = 0; i < TM; i++) {
        if (i >= t && i < T && A.m[i] == A.m[t]) {
          const z2 ai = i == t ? a : ahat_at_p(A, P, rr, U, i, f);
          const double w = zld(S, pidx(A, i, i, f)).x - (ai.x * ai.x + ai.y * ai.y);
          vals[2 + i] += w * lam;
          vals[2 + TM + i] += w;
          wsum += P->R[i * MTGP_MAXT + i] * w;
        }
      }
      const int64_t pos = A.col_off[c] + spec_pos(family, f, A.m[t]);
      if (family == FAM_DSEQ) {
        cols[pos] = (SR)wsum;
      } else {
        cols[2 * pos] = (SR)wsum;
        cols[2 * pos + 1] = (SR)0;
      }
    }
    for (int u = t + 1; u < T; u++) {
      const z2 au = ahat_at_p(A, P, rr, U, u, f & ((1ll << A.m[u]) - 1));
      const z2 wtu = zsub(zconj(zld(S, pidx(A, t, u, f))), zmulc(a, au));
      const double R2 = 2.0 * sqrt(ldexp(1.0, A.m[u] - A.m[t]));
      const int64_t pos = A.col_off[A.pc(t, u)] + spec_pos(family, f, A.m[t]);
      if (family == FAM_DSEQ) {
        cols[pos] = (SR)(R2 * wtu.x);
      } else {
        cols[2 * pos] = (SR)(R2 * wtu.x);
        cols[2 * pos + 1] = (SR)(-R2 * wtu.y);
      }
    }
  }
  block_sum_store<NQ>(vals, NQ, red, row);
}

}  // namespace mtgp

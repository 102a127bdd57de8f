// Gradient of the GCV loss at nested unequal sizes (Eq. MTGP_MLE_GCV_loss;
// the paper gives no gradient, this is the exact derivative):
//   dL_GCV = tr(W dLambda),
//   W = -(bhat ahat^H + ahat bhat^H) / s^2 + (2 q / s^3) Lambda^-2,
// ahat = Lambda^-1 rhat, bhat = Lambda^-2 rhat, q = |ahat|^2, s = tr Lambda^-1,
// needs Lambda^-2 on the sparsity pattern of Lambda, which the fill-free
// elimination's selected inverse does not give (Lambda^-1 is dense within a
// residue class).  With Lambda(e) = Lambda + e I, d/de Lambda(e)^-1 =
// -Lambda^-2: running the same elimination (task-order L D L^H, forward and
// backward substitution, selected inversion on the pattern) in dual numbers
// x + e x', with the pivot entries seeded with derivative 1, gives on the
// pattern Z = Lambda^-1 (value) and -Lambda^-2 (derivative), and for the
// right-hand sides ahat and -bhat, Lambda^-1 e_(u,0) and -Lambda^-2 e_(u,0)
// (the residue-0 unit solves of the GCV means, Eq. MTGP_optimal_tau).
// The derivative of an algorithm's output equals the derivative of the
// quantity it computes, so the derivative parts are exact up to rounding.
//
// Storage as the fill-free elimination (elim.hip), every entry a pair of
// complex numbers (value, derivative).
#include "kernels.h"

namespace mtgp {

namespace {

struct dr {
  double v, e;
};
struct dz {
  z2 v, e;
};

__device__ inline z2 cm(z2 a, z2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline z2 cmc(z2 a, z2 b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
__device__ inline z2 cadd2(z2 a, z2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline z2 csub2(z2 a, z2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline z2 cconj(z2 a) { return {a.x, -a.y}; }
__device__ inline z2 cscl(z2 a, double s) { return {a.x * s, a.y * s}; }

__device__ inline dz dmul(dz a, dz b) { return {cm(a.v, b.v), cadd2(cm(a.e, b.v), cm(a.v, b.e))}; }
// a conj(b)
__device__ inline dz dmulc(dz a, dz b) {
  return {cmc(a.v, b.v), cadd2(cmc(a.e, b.v), cmc(a.v, b.e))};
}
__device__ inline dz dadd(dz a, dz b) { return {cadd2(a.v, b.v), cadd2(a.e, b.e)}; }
__device__ inline dz dsub(dz a, dz b) { return {csub2(a.v, b.v), csub2(a.e, b.e)}; }
__device__ inline dz dconj(dz a) { return {cconj(a.v), cconj(a.e)}; }
__device__ inline dz dscl(dz a, dr s) {
  return {cscl(a.v, s.v), cadd2(cscl(a.e, s.v), cscl(a.v, s.e))};
}
__device__ inline dr dinv(dr d) {
  const double i = 1.0 / d.v;
  return {i, -d.e * i * i};
}
__device__ inline dr dre(dz a) { return {a.v.x, a.e.x}; }
__device__ inline dz dreal(dr a) { return {{a.v, 0.0}, {a.e, 0.0}}; }
__device__ inline dz dzero() { return {{0.0, 0.0}, {0.0, 0.0}}; }

__device__ inline int64_t gpidx(const Alg1Desc& A, int a, int b, int64_t g) {
  return A.so[a] + ((int64_t)(b - a) << A.m[a]) + g;
}

__device__ inline int gtask_of(const int64_t* off, int T, int64_t i) {
  int t = 0;
  while (t + 1 < T && i >= off[t + 1]) t++;
  return t;
}

// inverse-pattern entry between (u, g_u) and (v, g_v), u, v > t
__device__ inline dz gpair(const Alg1Desc& A, const dz* S, int u, int v, int64_t gu, int64_t gv) {
  if (u == v) return dreal(dre(S[gpidx(A, u, u, gu)]));
  if (u < v) return dconj(S[gpidx(A, u, v, gu)]);
  return S[gpidx(A, v, u, gv)];
}

__device__ inline double shfl_sum(double v, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

// Pattern values (diagonal derivative 1), yhat, unit right-hand sides.
template <typename SR>
__global__ void zd_init_kernel(const SR* __restrict__ cols, Alg1Desc A, const Params* __restrict__ P,
                               int family, int64_t N, const double* __restrict__ yhat,
                               dz* __restrict__ S, dz* __restrict__ rr, dz* __restrict__ U) {
  const int T = A.T;
  const int64_t nS = A.so[T], ms = A.msz[T - 1];
  const int64_t total = nS + N + (int64_t)T * ms;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nS) {
      const int a = gtask_of(A.so, T, i);
      const int64_t r = i - A.so[a];
      const int b = a + (int)(r >> A.m[a]);
      const int64_t g = r & ((1ll << A.m[a]) - 1);
      const z2 l = lam_at<SR>(cols, A, family, A.pc(a, b), g);
      if (b == a) {
        S[i] = {{P->R[a * MTGP_MAXT + a] * l.x + P->xi[a], 0.0}, {1.0, 0.0}};
      } else {
        const double sc = sqrt(ldexp(1.0, A.m[b] - A.m[a])) * P->R[a * MTGP_MAXT + b];
        S[i] = {cconj(cscl(l, sc)), {0.0, 0.0}};
      }
    } else if (i < nS + N) {
      const int64_t q = i - nS;
      const int t = gtask_of(A.task_off, T, q);
      const int64_t f = q - A.task_off[t];
      const int64_t yp = A.task_off[t] + spec_pos(family, f, A.m[t]);
      const z2 y = family == FAM_DSEQ ? z2{yhat[yp], 0.0} : z2{yhat[2 * yp], yhat[2 * yp + 1]};
      rr[q] = {y, {0.0, 0.0}};
    } else {
      const int64_t q = i - nS - N;
      const int64_t v = q / ms, node = q - v * ms;
      U[q] = {{node == A.coff[v] ? 1.0 : 0.0, 0.0}, {0.0, 0.0}};
    }
  }
}

// Stage t, later task u (the targets of the fill-free factorisation, each a
// sum of n_t / n_u terms over a group of G lanes).
__global__ __launch_bounds__(256) void zd_factor_kernel(Alg1Desc A, int t, int u, int G,
                                                        dz* __restrict__ S, dz* __restrict__ rr,
                                                        dz* __restrict__ U) {
  const int T = A.T;
  const int64_t nu = 1ll << A.m[u];
  const int64_t K = 1ll << (A.m[t] - A.m[u]);
  const int cs = A.m[T - 1];
  const int64_t cu = nu >> cs;
  const int64_t ms = A.msz[T - 1];
  const int64_t ntarget = (int64_t)(T - u) * nu + nu + (int64_t)T * cu;
  const int lane = threadIdx.x & (G - 1);
  const int64_t gstride = ((int64_t)gridDim.x * blockDim.x) / G;
  for (int64_t q = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
       q < ((ntarget + gstride - 1) / gstride) * gstride; q += gstride) {
    const bool live = q < ntarget;
    dz acc = dzero();
    int kind = 0, v = u;
    int64_t dst = 0;
    if (live) {
      int64_t g;
      if (q < (int64_t)(T - u) * nu) {
        v = u + (int)(q >> A.m[u]);
        g = q & (nu - 1);
        dst = gpidx(A, u, v, g);
        for (int64_t j = lane; j < K; j += G) {
          const int64_t f = g + (j << A.m[u]);
          const dr di = dinv(dre(S[gpidx(A, t, t, f)]));
          acc = dadd(acc, dscl(dmulc(S[gpidx(A, t, v, f)], S[gpidx(A, t, u, f)]), di));
        }
      } else if (q < (int64_t)(T - u) * nu + nu) {
        kind = 1;
        g = q - (int64_t)(T - u) * nu;
        dst = A.task_off[u] + g;
        for (int64_t j = lane; j < K; j += G) {
          const int64_t f = g + (j << A.m[u]);
          const dr di = dinv(dre(S[gpidx(A, t, t, f)]));
          acc = dadd(acc, dscl(dmul(S[gpidx(A, t, u, f)], rr[A.task_off[t] + f]), di));
        }
      } else {
        kind = 2;
        const int64_t r = q - (int64_t)(T - u) * nu - nu;
        const int rv = (int)(r / cu);
        const int64_t k = r - (int64_t)rv * cu;
        g = k << cs;
        dst = (int64_t)rv * ms + A.coff[u] + k;
        for (int64_t j = lane; j < K; j += G) {
          const int64_t f = g + (j << A.m[u]);
          const dr di = dinv(dre(S[gpidx(A, t, t, f)]));
          acc = dadd(acc, dscl(dmul(S[gpidx(A, t, u, f)],
                                    U[(int64_t)rv * ms + A.coff[t] + (f >> cs)]), di));
        }
      }
    }
    acc.v.x = shfl_sum(acc.v.x, G);
    acc.v.y = shfl_sum(acc.v.y, G);
    acc.e.x = shfl_sum(acc.e.x, G);
    acc.e.y = shfl_sum(acc.e.y, G);
    if (live && lane == 0) {
      if (kind == 0) {
        const dz s = dsub(S[dst], acc);
        S[dst] = v == u ? dreal(dre(s)) : s;
      } else if (kind == 1) {
        rr[dst] = dsub(rr[dst], acc);
      } else {
        U[dst] = dsub(U[dst], acc);
      }
    }
  }
}

// Backward stage t: right-hand sides and the selected inverse on the
// column of (t, f), written over it (values and derivatives).
template <int TM>
__global__ __launch_bounds__(256) void zd_back_kernel(Alg1Desc A, int t, dz* __restrict__ S,
                                                      dz* __restrict__ rr, dz* __restrict__ U,
                                                      int* __restrict__ status) {
  const int T = A.T;
  const int64_t nt = 1ll << A.m[t];
  const int cs = A.m[T - 1];
  const int64_t ms = A.msz[T - 1];
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nt;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = A.task_off[t] + f;
    const dr d = dre(S[gpidx(A, t, t, f)]);
    if (!(d.v > 0.0) || !isfinite(d.v)) flag_bad(status, node);
    const dr di = dinv(d);
    dz L[TM];
#pragma unroll
    for (int u = 0; u < TM; u++)
      L[u] = (u > t && u < T) ? dscl(S[gpidx(A, t, u, f)], di) : dzero();
    dz a = dscl(rr[node], di);
#pragma unroll
    for (int u = 0; u < TM; u++)
      if (u > t && u < T) a = dsub(a, dmulc(rr[A.task_off[u] + (f & ((1ll << A.m[u]) - 1))], L[u]));
    rr[node] = a;
    if ((f & ((1ll << cs) - 1)) == 0) {
      const int64_t k = f >> cs;
      for (int v = 0; v < T; v++) {
        dz* Uv = U + (int64_t)v * ms;
        dz b = dscl(Uv[A.coff[t] + k], di);
#pragma unroll
        for (int u = 0; u < TM; u++)
          if (u > t && u < T)
            b = dsub(b, dmulc(Uv[A.coff[u] + ((f & ((1ll << A.m[u]) - 1)) >> cs)], L[u]));
        Uv[A.coff[t] + k] = b;
      }
    }
    dz Zc[TM];
    dr ztt = di;
#pragma unroll
    for (int u = 0; u < TM; u++) {
      Zc[u] = dzero();
      if (u > t && u < T) {
        const int64_t gu = f & ((1ll << A.m[u]) - 1);
        dz acc = dzero();
#pragma unroll
        for (int v = 0; v < TM; v++)
          if (v > t && v < T)
            acc = dadd(acc, dmul(gpair(A, S, u, v, gu, f & ((1ll << A.m[v]) - 1)), L[v]));
        Zc[u] = {cscl(acc.v, -1.0), cscl(acc.e, -1.0)};
        const dr p = dre(dmulc(L[u], Zc[u]));  // Re(conj(Z_u) L_u)
        ztt.v -= p.v;
        ztt.e -= p.e;
      }
    }
    S[gpidx(A, t, t, f)] = dreal(ztt);
#pragma unroll
    for (int u = 0; u < TM; u++)
      if (u > t && u < T) S[gpidx(A, t, u, f)] = Zc[u];
  }
}

// GCV means from residue class 0 (one block): with the derivative parts
// -Lambda^-2 e_(u,0) and -Lambda^-2 yhat,
//   (E K^-2 E^T)_tu = sqrt(n_t n_u) (Lambda^-2)_{(t,0),(u,0)},
//   (E K^-2 y)_t = sqrt(n_t) (Lambda^-2 yhat)_(t,0)   (Eq. MTGP_optimal_tau).
__global__ void zd_tau_kernel(Alg1Desc A, Params* P, const dz* __restrict__ rr,
                              const dz* __restrict__ U) {
  __shared__ double M[MTGP_MAXT][MTGP_MAXT + 1];
  const int T = A.T;
  const int64_t ms = A.msz[T - 1];
  if (!A.profile) {
    if (threadIdx.x < T) P->tau_used[threadIdx.x] = P->tau[threadIdx.x];
    return;
  }
  for (int e = threadIdx.x; e < T * (T + 1); e += blockDim.x) {
    const int t = e / (T + 1), u = e - t * (T + 1);
    if (u < T)
      M[t][u] = -sqrt(ldexp(1.0, A.m[t] + A.m[u])) * U[(int64_t)u * ms + A.coff[t]].e.x;
    else
      M[t][T] = -sqrt(ldexp(1.0, A.m[t])) * rr[A.task_off[t]].e.x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < T; c++) {  // Gaussian elimination with partial pivoting
      int pv = c;
      for (int i = c + 1; i < T; i++)
        if (fabs(M[i][c]) > fabs(M[pv][c])) pv = i;
      for (int k = 0; k <= T; k++) {
        const double tmp = M[c][k];
        M[c][k] = M[pv][k];
        M[pv][k] = tmp;
      }
      for (int i = c + 1; i < T; i++) {
        const double fct = M[i][c] / M[c][c];
        for (int k = c; k <= T; k++) M[i][k] -= fct * M[c][k];
      }
    }
    double tau[MTGP_MAXT];
    for (int c = T - 1; c >= 0; c--) {
      double acc = M[c][T];
      for (int k = c + 1; k < T; k++) acc -= M[c][k] * tau[k];
      tau[c] = acc / M[c][c];
    }
    for (int c = 0; c < T; c++) P->tau_used[c] = tau[c];
  }
}

namespace {
// ahat (value) and bhat (from the derivative) of node (u, g) for the means
// used: the data solutions minus the unit solutions on residue class 0
__device__ inline void gcv_ab(const Alg1Desc& A, const Params* P, const dz* rr, const dz* U, int u,
                              int64_t g, z2& a, z2& b) {
  const dz x = rr[A.task_off[u] + g];
  a = x.v;
  b = cscl(x.e, -1.0);
  const int cs = A.m[A.T - 1];
  if ((g & ((1ll << cs) - 1)) == 0) {
    const int64_t ms = A.msz[A.T - 1];
    const int64_t k = A.coff[u] + (g >> cs);
    for (int v = 0; v < A.T; v++) {
      const double c = sqrt(ldexp(1.0, A.m[v])) * P->tau_used[v];
      const dz e = U[(int64_t)v * ms + k];
      a = csub2(a, cscl(e.v, c));
      b = cadd2(b, cscl(e.e, c));
    }
  }
}
}  // namespace

// Final pass over all nodes.  WEIGHTS = false: q = |ahat|^2 and s = tr
// Lambda^-1 (slots 0 and 1).  WEIGHTS = true (q and s in P from the first
// pass): the same sums, Re bhat_t(0) / s^2 in the mean slots (dL/dtau_t =
// -2 sqrt(n_t) Re bhat_t(0) / s^2), and W written over the spectrum as the
// MLE elimination writes its weights (pair column (t, u), t < u, at f:
// 2 sqrt(n_u / n_t) conj(W_{(t,f),(u,f mod n_u)}); diagonal column: sum over
// the tasks of that length of R_tt W_tt), with G_tt and sum W_tt.
template <typename SR, int TM, bool WEIGHTS>
__global__ __launch_bounds__(256) void zd_final_kernel(SR* __restrict__ cols, Alg1Desc A, int64_t N,
                                                       const Params* __restrict__ P, int family,
                                                       const dz* __restrict__ S,
                                                       const dz* __restrict__ rr,
                                                       const dz* __restrict__ U,
                                                       double* __restrict__ partials) {
  constexpr int NQ = 2 + 3 * TM;
  __shared__ double red[4 * NQ];
  const int T = A.T;
  double vals[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) vals[q] = 0.0;
  const double sg = WEIGHTS ? P->gcv_s : 1.0, qg = WEIGHTS ? P->gcv_q : 0.0;
  const double c1 = -1.0 / (sg * sg), c2 = 2.0 * qg / (sg * sg * sg);
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < N;
       node += (int64_t)gridDim.x * blockDim.x) {
    const int t = gtask_of(A.task_off, T, node);
    const int64_t f = node - A.task_off[t];
    z2 a, b;
    gcv_ab(A, P, rr, U, t, f, a, b);
    vals[0] += a.x * a.x + a.y * a.y;
    vals[1] += S[gpidx(A, t, t, f)].v.x;
    if (!WEIGHTS) continue;
    if (f == 0) {
#pragma unroll
      for (int i = 0; i < TM; i++)
        if (i == t) vals[2 + 2 * TM + i] = b.x / (sg * sg);
    }
    if (A.df(t) == t) {
      const int c = A.pc(t, t);
      const double lam = lam_at<SR>(cols, A, family, c, f).x;
      double wsum = 0.0;
#pragma unroll
      for (int i = 0; i < TM; i++) {
        if (i >= t && i < T && A.m[i] == A.m[t]) {
          z2 ai = a, bi = b;
          if (i != t) gcv_ab(A, P, rr, U, i, f, ai, bi);
          const double z2ii = -S[gpidx(A, i, i, f)].e.x;  // (Lambda^-2)_ii
          const double w = c1 * 2.0 * (bi.x * ai.x + bi.y * ai.y) + c2 * z2ii;
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
      z2 au, bu;
      gcv_ab(A, P, rr, U, u, f & ((1ll << A.m[u]) - 1), au, bu);
      // (Lambda^-2)_{(t,f),(u,.)} = conj of the stored (u,.),(t,f) entry, negated
      const z2 z2tu = cscl(cconj(S[gpidx(A, t, u, f)].e), -1.0);
      const z2 wtu = cadd2(cscl(cadd2(cmc(b, au), cmc(a, bu)), c1), cscl(z2tu, c2));
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
  block_sum_store<NQ>(vals, NQ, red, partials + (size_t)blockIdx.x * NQ);
}

namespace {
unsigned gcv_grid(int64_t work) {
  const int64_t b = (work + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}
}  // namespace

// Elimination in dual numbers, GCV means and the first pass (q, s); the
// second pass (weights) runs after the loss values are in P.
template <typename SR>
int launch_zerofill_gcv_dual(SR* cols, const Alg1Desc& A1, int64_t N, Params* P, int family,
                             const double* yhat, void* buf, double* partials, int* status,
                             bool weights, hipStream_t st) {
  const int T = A1.T;
  const int64_t ms = A1.msz[T - 1];
  dz* S = static_cast<dz*>(buf);
  dz* rr = S + A1.so[T];
  dz* U = rr + N;
  const dim3 fgrid((unsigned)zf_final_blocks(N));
#define MTGP_ZDF(TMV, W)                                                                        \
  hipLaunchKernelGGL((zd_final_kernel<SR, TMV, W>), fgrid, dim3(256), 0, st, cols, A1, N, P,    \
                     family, S, rr, U, partials)
#define MTGP_ZDF_T(W)            \
  do {                           \
    if (T <= 1) MTGP_ZDF(1, W);  \
    else if (T <= 2) MTGP_ZDF(2, W); \
    else if (T <= 4) MTGP_ZDF(4, W); \
    else if (T <= 8) MTGP_ZDF(8, W); \
    else MTGP_ZDF(16, W);        \
  } while (0)
  if (weights) {
    MTGP_ZDF_T(true);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  hipLaunchKernelGGL(zd_init_kernel<SR>, dim3(gcv_grid(A1.so[T] + N + (int64_t)T * ms)), dim3(256),
                     0, st, cols, A1, P, family, N, yhat, S, rr, U);
  const int cs = A1.m[T - 1];
  for (int t = 0; t + 1 < T; t++) {
    for (int u = t + 1; u < T; u++) {
      const int64_t nu = 1ll << A1.m[u];
      const int64_t K = 1ll << (A1.m[t] - A1.m[u]);
      const int G = K >= 64 ? 64 : (int)K;
      const int64_t ntarget = (int64_t)(T - u) * nu + nu + (int64_t)T * (nu >> cs);
      hipLaunchKernelGGL(zd_factor_kernel, dim3(gcv_grid(ntarget * G)), dim3(256), 0, st, A1, t,
                         u, G, S, rr, U);
    }
  }
  for (int t = T - 1; t >= 0; t--) {
    const dim3 g(gcv_grid((int64_t)1 << A1.m[t]));
    if (T <= 1) hipLaunchKernelGGL(zd_back_kernel<1>, g, dim3(256), 0, st, A1, t, S, rr, U, status);
    else if (T <= 2) hipLaunchKernelGGL(zd_back_kernel<2>, g, dim3(256), 0, st, A1, t, S, rr, U, status);
    else if (T <= 4) hipLaunchKernelGGL(zd_back_kernel<4>, g, dim3(256), 0, st, A1, t, S, rr, U, status);
    else if (T <= 8) hipLaunchKernelGGL(zd_back_kernel<8>, g, dim3(256), 0, st, A1, t, S, rr, U, status);
    else hipLaunchKernelGGL(zd_back_kernel<16>, g, dim3(256), 0, st, A1, t, S, rr, U, status);
  }
  hipLaunchKernelGGL(zd_tau_kernel, dim3(1), dim3(256), 0, st, A1, P, rr, U);
  MTGP_ZDF_T(false);
#undef MTGP_ZDF_T
#undef MTGP_ZDF
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_zerofill_gcv_dual<double>(double*, const Alg1Desc&, int64_t, Params*, int,
                                              const double*, void*, double*, int*, bool,
                                              hipStream_t);
template int launch_zerofill_gcv_dual<float>(float*, const Alg1Desc&, int64_t, Params*, int,
                                             const double*, void*, double*, int*, bool,
                                             hipStream_t);

}  // namespace mtgp

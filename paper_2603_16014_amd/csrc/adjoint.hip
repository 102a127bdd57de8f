// Adjoint pass of the digital-sequence path: dispatch by kernel type of the
// low-bit adjoint transform fused with the derivative reduction (the kernel
// and the adjoint identity it evaluates are in fused_eval.h).
#include "kernels.h"

namespace mtgp {

template <typename Real, typename TIn>
int launch_adj_reduce(const TIn* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                      const uint32_t* colshift, const Params* P, const KDesc& kd, double* partials,
                      const Sched& sc, hipStream_t st, int run) {
  if (ncols <= 0) return 0;
  switch (kt_of(kd.family, kd.order, kd.adaptive)) {
    case KT_DSI1:
      return launch_adj_reduce_kt<Real, TIn, KT_DSI1>(base, col_stride, ncols, m, gen, colshift,
                                                      P, kd.d, partials, sc, st, run);
    case KT_DSI2:
      return launch_adj_reduce_kt<Real, TIn, KT_DSI2>(base, col_stride, ncols, m, gen, colshift,
                                                      P, kd.d, partials, sc, st, run);
    case KT_DSI3:
      return launch_adj_reduce_kt<Real, TIn, KT_DSI3>(base, col_stride, ncols, m, gen, colshift,
                                                      P, kd.d, partials, sc, st, run);
    case KT_DSI4:
      return launch_adj_reduce_kt<Real, TIn, KT_DSI4>(base, col_stride, ncols, m, gen, colshift,
                                                      P, kd.d, partials, sc, st, run);
    case KT_DSIA:
      return launch_adj_reduce_kt<Real, TIn, KT_DSIA>(base, col_stride, ncols, m, gen, colshift,
                                                      P, kd.d, partials, sc, st, run);
    default: return -1;
  }
}

template int launch_adj_reduce<double, double>(const double*, int64_t, int, int, const uint32_t*,
                                               const uint32_t*, const Params*, const KDesc&,
                                               double*, const Sched&, hipStream_t, int);
template int launch_adj_reduce<double, float>(const float*, int64_t, int, int, const uint32_t*,
                                              const uint32_t*, const Params*, const KDesc&,
                                              double*, const Sched&, hipStream_t, int);
template int launch_adj_reduce<float, float>(const float*, int64_t, int, int, const uint32_t*,
                                             const uint32_t*, const Params*, const KDesc&,
                                             double*, const Sched&, hipStream_t, int);

}  // namespace mtgp

// Instantiations of the fused low-bit adjoint pass + derivative reduction for one
// kernel type (KT_DSI4); split per type so the kernels compile in parallel.
#include "fused_eval.h"

namespace mtgp {
template int launch_adj_reduce_kt<double, double, KT_DSI4>(const double*, int64_t, int, int,
    const uint32_t*, const uint32_t*, const Params*, int, double*, const Sched&, hipStream_t, int);
template int launch_adj_reduce_kt<double, float, KT_DSI4>(const float*, int64_t, int, int,
    const uint32_t*, const uint32_t*, const Params*, int, double*, const Sched&, hipStream_t, int);
template int launch_adj_reduce_kt<float, float, KT_DSI4>(const float*, int64_t, int, int,
    const uint32_t*, const uint32_t*, const Params*, int, double*, const Sched&, hipStream_t, int);
}  // namespace mtgp

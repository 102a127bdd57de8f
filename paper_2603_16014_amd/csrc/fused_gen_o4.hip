// Instantiations of the fused column generation + low-bit forward pass for one
// kernel type (KT_DSI4); split per type so the kernels compile in parallel.
#include "fused_eval.h"

namespace mtgp {
template int launch_gen_fwd_kt<double, double, KT_DSI4>(double*, int64_t, int, int, const uint32_t*,
    const uint32_t*, const Params*, int, const Sched&, hipStream_t);
template int launch_gen_fwd_kt<double, float, KT_DSI4>(float*, int64_t, int, int, const uint32_t*,
    const uint32_t*, const Params*, int, const Sched&, hipStream_t);
template int launch_gen_fwd_kt<float, float, KT_DSI4>(float*, int64_t, int, int, const uint32_t*,
    const uint32_t*, const Params*, int, const Sched&, hipStream_t);
}  // namespace mtgp

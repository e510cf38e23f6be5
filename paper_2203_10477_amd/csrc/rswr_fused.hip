// rswr_fused.hip -- dispatch of the fused span launch to its kind (the
// kernels are instantiated in rswr_fused_plain.hip, rswr_fused_ext_*.hip
// and rswr_fused_gen.hip).
#include "rswr_internal.h"

namespace rswr {

template <typename T>
hipError_t launch_fused(const UpdateArgs<T>& a, int threads, int per_thread, int kind,
                        hipStream_t s) {
  if (kind == kFusedGeneral)
    return launch_fused_kind<T, kFusedGeneral>(a, threads, per_thread, s);
  if (kind == kFusedExt) return launch_fused_kind<T, kFusedExt>(a, threads, per_thread, s);
  return launch_fused_kind<T, kFusedPlain>(a, threads, per_thread, s);
}

template hipError_t launch_fused<float>(const UpdateArgs<float>&, int, int, int,
                                        hipStream_t);
template hipError_t launch_fused<double>(const UpdateArgs<double>&, int, int, int,
                                         hipStream_t);

}  // namespace rswr

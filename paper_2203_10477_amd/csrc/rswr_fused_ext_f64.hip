// rswr_fused_ext_f64.hip -- instantiation of the fused span kernel, launch kind
// kFusedExt (double).
#include "rswr_fused_kernel.h"

namespace rswr {

template hipError_t launch_fused_kind<double, kFusedExt>(const UpdateArgs<double>&, int, int,
                                                      hipStream_t);

}  // namespace rswr

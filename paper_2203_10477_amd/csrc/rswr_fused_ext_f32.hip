// rswr_fused_ext_f32.hip -- instantiation of the fused span kernel, launch kind
// kFusedExt (float).
#include "rswr_fused_kernel.h"

namespace rswr {

template hipError_t launch_fused_kind<float, kFusedExt>(const UpdateArgs<float>&, int, int,
                                                      hipStream_t);

}  // namespace rswr

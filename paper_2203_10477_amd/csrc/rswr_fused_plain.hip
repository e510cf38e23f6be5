// rswr_fused_plain.hip -- instantiation of the fused span kernel, launch kind
// kFusedPlain (float and double).
#include "rswr_fused_kernel.h"

namespace rswr {

template hipError_t launch_fused_kind<float, kFusedPlain>(const UpdateArgs<float>&, int, int,
                                                      hipStream_t);
template hipError_t launch_fused_kind<double, kFusedPlain>(const UpdateArgs<double>&, int, int,
                                                      hipStream_t);

}  // namespace rswr

// rswr_fused_gen.hip -- instantiation of the fused span kernel, launch kind
// kFusedGeneral (float and double).
#include "rswr_fused_kernel.h"

namespace rswr {

template hipError_t launch_fused_kind<float, kFusedGeneral>(const UpdateArgs<float>&, int, int,
                                                      hipStream_t);
template hipError_t launch_fused_kind<double, kFusedGeneral>(const UpdateArgs<double>&, int, int,
                                                      hipStream_t);

}  // namespace rswr

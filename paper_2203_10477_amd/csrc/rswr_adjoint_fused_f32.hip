// rswr_adjoint_fused_f32.hip -- the fused adjoint update (FP32): tiles
// that hold an input end advance its W frame themselves (rswr_adjoint.h).
#include "rswr_adjoint.h"

namespace rswr {

template hipError_t launch_adj_update_kind<float, true>(const AdjUpdateArgs<float>&, int, int,
                                                        bool, hipStream_t);
template bool adj_update_fused_fits<float>(int, int);

}  // namespace rswr

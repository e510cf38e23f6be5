// rswr_adjoint_fused_f64.hip -- the fused adjoint update (FP64): tiles
// that hold an input end advance its W frame themselves (rswr_adjoint.h).
#include "rswr_adjoint.h"

namespace rswr {

template hipError_t launch_adj_update_kind<double, true>(const AdjUpdateArgs<double>&, int, int,
                                                         bool, hipStream_t);
template bool adj_update_fused_fits<double>(int, int);

}  // namespace rswr

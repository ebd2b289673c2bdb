// Instantiations of the 2D stage kernel for the P_ACC64 arithmetic mode.
#include "stage2d.h"

namespace hweno {

hipError_t launch_stage2d_acc64(int flux, int Q, int mode, int variant, const StageArgs& a,
                             int grid, hipStream_t s) {
    return stage2d_launch_prec<P_ACC64>(flux, Q, mode, variant, a, grid, s);
}

}  // namespace hweno

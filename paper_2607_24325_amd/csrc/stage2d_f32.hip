// Instantiations of the 2D stage kernel for the P_F32 arithmetic mode.
#include "stage2d.h"

namespace hweno {

hipError_t launch_stage2d_f32(int flux, int Q, int mode, int variant, const StageArgs& a,
                             int grid, hipStream_t s) {
    return stage2d_launch_prec<P_F32>(flux, Q, mode, variant, a, grid, s);
}

}  // namespace hweno

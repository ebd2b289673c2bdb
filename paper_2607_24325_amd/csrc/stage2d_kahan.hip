// Instantiations of the 2D stage kernel for the P_KAHAN arithmetic mode.
#include "stage2d.h"

namespace hweno {

hipError_t launch_stage2d_kahan(int flux, int Q, int mode, const StageArgs& a, int grid,
                              hipStream_t s) {
    if (flux == F_EULER) {
        if (Q == 2) stage2d_kernel<P_KAHAN, 4, 2, F_EULER><<<grid, 256, 0, s>>>(a, mode);
        else stage2d_kernel<P_KAHAN, 4, 3, F_EULER><<<grid, 256, 0, s>>>(a, mode);
    } else if (flux == F_BURGERS) {
        if (Q == 2) stage2d_kernel<P_KAHAN, 1, 2, F_BURGERS><<<grid, 64, 0, s>>>(a, mode);
        else stage2d_kernel<P_KAHAN, 1, 3, F_BURGERS><<<grid, 64, 0, s>>>(a, mode);
    } else {
        if (Q == 2) stage2d_kernel<P_KAHAN, 1, 2, F_ADV><<<grid, 64, 0, s>>>(a, mode);
        else stage2d_kernel<P_KAHAN, 1, 3, F_ADV><<<grid, 64, 0, s>>>(a, mode);
    }
    return hipGetLastError();
}

}  // namespace hweno

// Instantiations and launcher of the 1D stage kernel.
#include "stage1d.h"

namespace hweno {

template <int P>
static hipError_t dispatch1d(int flux, int mode, const StageArgs& a, int grid, hipStream_t s) {
    if (flux == F_ADV) stage1d_kernel<P, 1, F_ADV><<<grid, 256, 0, s>>>(a, mode);
    else if (flux == F_BURGERS) stage1d_kernel<P, 1, F_BURGERS><<<grid, 256, 0, s>>>(a, mode);
    else stage1d_kernel<P, 3, F_EULER><<<grid, 256, 0, s>>>(a, mode);
    return hipGetLastError();
}

hipError_t launch_stage1d(int prec, int flux, int mode, const StageArgs& a, int grid,
                          hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (grid <= 0 || grid > a.ntiles) grid = a.ntiles;
    if (prec == P_F64) return dispatch1d<P_F64>(flux, mode, a, grid, s);
    if (prec == P_F32) return dispatch1d<P_F32>(flux, mode, a, grid, s);
    if (prec == P_ACC64) return dispatch1d<P_ACC64>(flux, mode, a, grid, s);
    if (prec == P_KAHAN) return dispatch1d<P_KAHAN>(flux, mode, a, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace hweno

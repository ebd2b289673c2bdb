// Instantiations and launcher of the 1D stage kernel.
#include "stage1d.h"

namespace hweno {

template <int P, int K, int FLUX, bool CH = false>
static void launch_modes(int mode, const StageArgs& a, int grid, hipStream_t s) {
    switch (mode) {
        case MODE_RHS: stage1d_kernel<P, K, FLUX, MODE_RHS, CH><<<grid, 256, 0, s>>>(a); break;
        case MODE_S1: stage1d_kernel<P, K, FLUX, MODE_S1, CH><<<grid, 256, 0, s>>>(a); break;
        case MODE_S2: stage1d_kernel<P, K, FLUX, MODE_S2, CH><<<grid, 256, 0, s>>>(a); break;
        default: stage1d_kernel<P, K, FLUX, MODE_S3, CH><<<grid, 256, 0, s>>>(a); break;
    }
}

template <int P>
static hipError_t dispatch1d(int flux, int mode, const StageArgs& a, int grid, hipStream_t s) {
    if (flux == F_ADV) launch_modes<P, 1, F_ADV>(mode, a, grid, s);
    else if (flux == F_BURGERS) launch_modes<P, 1, F_BURGERS>(mode, a, grid, s);
    else if (a.sch.charwise) launch_modes<P, 3, F_EULER, true>(mode, a, grid, s);
    else launch_modes<P, 3, F_EULER>(mode, a, grid, s);
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

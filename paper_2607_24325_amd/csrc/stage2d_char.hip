// Instantiations and launcher of the 2D characteristic-variable stage kernel
// (Euler only).
#include "stage2d_char.h"

namespace hweno {

template <int P, int Q>
static void launch_modes(int mode, const StageArgs& a, int grid, hipStream_t s) {
    switch (mode) {
        case MODE_RHS: stage2d_char_kernel<P, Q, MODE_RHS><<<grid, 256, 0, s>>>(a); break;
        case MODE_S1: stage2d_char_kernel<P, Q, MODE_S1><<<grid, 256, 0, s>>>(a); break;
        case MODE_S2: stage2d_char_kernel<P, Q, MODE_S2><<<grid, 256, 0, s>>>(a); break;
        default: stage2d_char_kernel<P, Q, MODE_S3><<<grid, 256, 0, s>>>(a); break;
    }
}

template <int P>
static void launch_q(int Q, int mode, const StageArgs& a, int grid, hipStream_t s) {
    if (Q == 2) launch_modes<P, 2>(mode, a, grid, s);
    else launch_modes<P, 3>(mode, a, grid, s);
}

hipError_t launch_stage2d_char(int prec, int Q, int mode, const StageArgs& a, int grid,
                               hipStream_t s) {
    if (prec == P_F64) launch_q<P_F64>(Q, mode, a, grid, s);
    else if (prec == P_F32) launch_q<P_F32>(Q, mode, a, grid, s);
    else if (prec == P_ACC64) launch_q<P_ACC64>(Q, mode, a, grid, s);
    else if (prec == P_KAHAN) launch_q<P_KAHAN>(Q, mode, a, grid, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace hweno

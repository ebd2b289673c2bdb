// Instantiations of the 2D stage kernel for the P_ACC64 arithmetic mode.
#include "stage2d.h"

namespace hweno {

template <int K, int Q, int FLUX>
static void launch_modes(int mode, const StageArgs& a, int grid, hipStream_t s) {
    constexpr int threads = 64 * K;
    switch (mode) {
        case MODE_RHS: stage2d_kernel<P_ACC64, K, Q, FLUX, MODE_RHS><<<grid, threads, 0, s>>>(a); break;
        case MODE_S1: stage2d_kernel<P_ACC64, K, Q, FLUX, MODE_S1><<<grid, threads, 0, s>>>(a); break;
        case MODE_S2: stage2d_kernel<P_ACC64, K, Q, FLUX, MODE_S2><<<grid, threads, 0, s>>>(a); break;
        default: stage2d_kernel<P_ACC64, K, Q, FLUX, MODE_S3><<<grid, threads, 0, s>>>(a); break;
    }
}

hipError_t launch_stage2d_acc64(int flux, int Q, int mode, const StageArgs& a, int grid,
                              hipStream_t s) {
    if (flux == F_EULER) {
        if (Q == 2) launch_modes<4, 2, F_EULER>(mode, a, grid, s);
        else launch_modes<4, 3, F_EULER>(mode, a, grid, s);
    } else if (flux == F_BURGERS) {
        if (Q == 2) launch_modes<1, 2, F_BURGERS>(mode, a, grid, s);
        else launch_modes<1, 3, F_BURGERS>(mode, a, grid, s);
    } else {
        if (Q == 2) launch_modes<1, 2, F_ADV>(mode, a, grid, s);
        else launch_modes<1, 3, F_ADV>(mode, a, grid, s);
    }
    return hipGetLastError();
}

}  // namespace hweno

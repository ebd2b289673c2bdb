// Launcher of the 2D stage kernel (instantiations live in stage2d_<mode>.hip).
#include "internal.h"

namespace hweno {

hipError_t launch_stage2d_f64(int flux, int Q, int mode, int variant, const StageArgs& a, int grid,
                             hipStream_t s);
hipError_t launch_stage2d_f32(int flux, int Q, int mode, int variant, const StageArgs& a, int grid,
                             hipStream_t s);
hipError_t launch_stage2d_acc64(int flux, int Q, int mode, int variant, const StageArgs& a, int grid,
                             hipStream_t s);
hipError_t launch_stage2d_kahan(int flux, int Q, int mode, int variant, const StageArgs& a, int grid,
                             hipStream_t s);
hipError_t launch_stage2d_char(int prec, int Q, int mode, const StageArgs& a, int grid, hipStream_t s);

hipError_t launch_stage2d(int prec, int flux, int Q, int mode, int variant, const StageArgs& a,
                          int grid, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (grid <= 0 || grid > a.ntiles) grid = a.ntiles;
    if (a.sch.charwise && flux == F_EULER) return launch_stage2d_char(prec, Q, mode, a, grid, s);
    if (prec == P_F64) return launch_stage2d_f64(flux, Q, mode, variant, a, grid, s);
    if (prec == P_F32) return launch_stage2d_f32(flux, Q, mode, variant, a, grid, s);
    if (prec == P_ACC64) return launch_stage2d_acc64(flux, Q, mode, variant, a, grid, s);
    if (prec == P_KAHAN) return launch_stage2d_kahan(flux, Q, mode, variant, a, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace hweno

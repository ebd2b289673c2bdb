// Internal definitions shared by the host runtime and the HIP kernels of
// libhweno (gfx950).  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hweno.h"

namespace hweno {

// Arithmetic modes (values match HWENO_F64 ... HWENO_F32_KAHAN).
enum Prec : int { P_F64 = 0, P_F32 = 1, P_ACC64 = 2, P_KAHAN = 3 };
enum FluxKind : int { F_ADV = 0, F_BURGERS = 1, F_EULER = 2 };
enum SmoothnessKind : int { BETA_MOMENT = 0, BETA_CLASSICAL = 1 };
enum BC : int { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2 };
enum WeightMode : int { W_PAPER = 0, W_BETA = 1, W_BETA2 = 2, W_LINEAR = 3 };

// What a stage launch computes.
//   MODE_RHS: L(U) and U-hat of the input set, written as doubles;
//   MODE_S1 : U1 = Uhat^n + dt L(U^n), saves the hats of U^n;
//   MODE_S2 : U2 = 3/4 Uhat^n + 1/4 (Uhat1 + dt L(U1));
//   MODE_S3 : U^{n+1} = 1/3 Uhat^n + 2/3 (Uhat2 + dt L(U2)), written over U^n.
enum Mode : int { MODE_RHS = 0, MODE_S1 = 1, MODE_S2 = 2, MODE_S3 = 3 };

// Per-problem table, resident in device memory.
struct ProbDev {
    int32_t nx, ny, bc_x, bc_y;
    int64_t off_u;  // element offset of the problem's K u-bar planes
    int64_t off_d;  // element offset of its K*D derivative planes
    double dx, dy, inv_dx, inv_dy;
    double dxe, dye;   // dx^e, dy^e of the time-step rule
    double t, t_end;
    double dt;         // step being taken (0 when inactive)
    double dt_in;      // requested step when the caller supplies one
    uint64_t ax_bits;  // max wave speeds of the current state, as the bits of
    uint64_t ay_bits;  // non-negative doubles
    uint64_t ax_next;  // the same for the state stage 3 is writing
    uint64_t ay_next;
    int32_t active;    // 1 while the current step advances this problem
    int32_t last;      // the current step lands exactly on t_end
    int32_t err;       // non-admissible state seen: ERR_STATE_BAD (a stored state),
                       // ERR_STAGE_BAD (an intermediate stage input)
    int32_t alpha_valid;  // ax_bits/ay_bits hold the speeds of the current state
    int64_t bad_cell;  // smallest flat index of a non-admissible cell
};

// Global step control, resident in device memory.
struct StepCtl {
    double cfl;
    int32_t use_dt_in;
    int32_t nprob;
    int32_t dim;
    int32_t nactive;   // problems still short of t_end after the last step
    int32_t step_active;  // some problem advanced in the current step
    int32_t pad;
    int64_t steps;     // steps in which some problem advanced
};

// 2D tile: a strip of 64 loaded columns (60 output columns starting at i0)
// marching through rows j0 .. j0+nrows-1.
struct Tile2D {
    int32_t prob, i0, j0, nrows;
};

// 1D tile: 254 output cells starting at c0.
struct Tile1D {
    int32_t prob, c0;
};

// Reduction chunk: cells [start, start+count) of one problem.
struct Chunk {
    int32_t prob, start, count, pad;
};

constexpr int STRIP_OUT = 60;      // output columns per 2D strip (64 lanes - 4 halo)
constexpr int TILE1D_OUT = 254;    // output cells per 1D tile (256 threads - 2)
constexpr int CHUNK_CELLS = 2048;  // cells per reduction chunk

// Scheme constants of one handle.
struct Scheme {
    double gam[5];     // linear weights gamma_0..gamma_M
    double eps;
    double gas_gamma;
    double adv[2];
    int32_t weights;   // WeightMode
    int32_t Q;         // Gauss points per edge (2D)
    int32_t charwise;  // Euler: reconstruct in local characteristic variables
    int32_t smoothness;   // SmoothnessKind of p0's indicator
};

// Buffers of one state set in the internal layout.
struct StateBuf {
    void* u;  // K u-bar planes per problem (double, float, or float2 for Kahan)
    void* d;  // K*D derivative planes per problem
};

struct StageArgs {
    StateBuf in;        // U^(k): stencil input
    StateBuf out;       // U^(k+1)
    const void* un;     // u-bar of U^n (stages 2, 3)
    void* h;            // saved hats of U^n
    double* L_out;      // MODE_RHS outputs (boundary layout, double)
    double* Uh_out;
    ProbDev* probs;
    const void* tiles;
    int32_t ntiles;
    int32_t tile_offset;
    Scheme sch;
};

// --- launchers (defined in the .hip files) ------------------------------
hipError_t launch_stage1d(int prec, int flux, int mode, const StageArgs& a, int grid,
                          hipStream_t s);
// variant: register variant of the Euler stage kernels (0 or 1; see
// stage2d_min_blocks), ignored for the scalar laws and the characteristic
// kernel.
hipError_t launch_stage2d(int prec, int flux, int Q, int mode, int variant, const StageArgs& a,
                          int grid, hipStream_t s);
// all_problems: zero the speeds of every problem (queries), or only of those
// whose speeds are not current (time stepping).
// Which problems a speed reset / reduction covers: every problem (after
// set_state), those whose speeds are not current (step start), or those
// active in the step (the per-stage speeds of stages 2 and 3).
enum SpeedSel : int { SEL_STALE = 0, SEL_ALL = 1, SEL_ACTIVE = 2 };
constexpr int ERR_STATE_BAD = 1, ERR_STAGE_BAD = 2;
hipError_t launch_reset(ProbDev* probs, StepCtl* ctl, int nprob, int sel, hipStream_t s);
// all_problems: 1 = every problem (rhs / alpha queries); 0 = only problems
// still short of t_end, without a pending error and whose speeds are not
// current (time stepping: stage 3 computes them for the next step).
hipError_t launch_alpha(int prec, int flux, int dim, const void* u, ProbDev* probs,
                        const Chunk* chunks, int nchunks, const Scheme& sch, int sel,
                        int grid, hipStream_t s);
hipError_t launch_dt(ProbDev* probs, StepCtl* ctl, int nprob, int use_dt_in, int own_ctl,
                     hipStream_t s);
hipError_t launch_finish(ProbDev* probs, StepCtl* ctl, int nprob, hipStream_t s);
// Converts one problem's state between the boundary layout (double,
// ext[((var*K + c)*ny + j)*nx + i]) and the internal planes of buf.
hipError_t launch_pack(int prec, int to_internal, double* ext, StateBuf buf, int64_t off_u,
                       int64_t off_d, int K, int nvar, int64_t ncell, hipStream_t s);

// --- host helpers of the C ABI (api.cpp) --------------------------------
// Checks problems and configuration (ERR_ARG with the reason as the
// thread's last error).
int validate_problems(const hweno_problem* probs, int32_t nprob, const hweno_config* cfg);
// Sets the thread's last error (hweno_last_error(NULL)); returns code.
int thread_error(int code, const char* fmt, ...);
Scheme scheme_of(const hweno_problem& p0, const hweno_config& cfg);
// Per-problem table entry (static fields; time 0, speeds unknown).
ProbDev probdev_of(const hweno_problem& pr, const hweno_config& cfg, int64_t off_u,
                   int64_t off_d);

}  // namespace hweno

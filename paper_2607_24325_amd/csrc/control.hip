// Per-step control kernels: wave-speed reduction for the global
// Lax-Friedrichs flux and the CFL rule, time-step selection, time update,
// and conversion between the boundary layout and the internal planes.
#include "device_common.h"

namespace hweno {

// Zeroes the wave-speed maxima that are about to be recomputed (SpeedSel)
// and, at the start of a step, the step counters.
__global__ void reset_kernel(ProbDev* probs, StepCtl* ctl, int nprob, int sel) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) {
        const ProbDev& P_ = probs[p];
        const bool pick = sel == SEL_ALL || (sel == SEL_STALE && !P_.alpha_valid) ||
                          (sel == SEL_ACTIVE && P_.active && !(P_.err & ERR_STAGE_BAD));
        if (pick) {
            probs[p].ax_bits = 0;
            probs[p].ay_bits = 0;
        }
    }
    if (p == 0 && sel != SEL_ACTIVE) {
        ctl->nactive = 0;
        ctl->step_active = 0;
    }
}

// alpha_x = max |f'(u)|, alpha_y = max |g'(u)| over the cell averages of a
// problem (Euler: |velocity| + sound speed), in double precision; cells that
// are not finite or have rho <= 0 / p <= 0 flag the problem.
template <int P, int FLUX, int DIM>
__global__ void __launch_bounds__(256) alpha_kernel(const void* uptr, ProbDev* probs,
                                                    const Chunk* chunks, int nchunks,
                                                    Scheme sch, int sel) {
    using TU = typename PrecT<P>::TU;
    constexpr int K = FLUX == F_EULER ? (DIM == 1 ? 3 : 4) : 1;
    __shared__ double smx[4], smy[4];
    __shared__ long long sbad[4];
    const TU* U = (const TU*)uptr;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const Chunk chunk = chunks[ch];
        ProbDev& P_ = probs[chunk.prob];
        if (sel == SEL_STALE && (!(P_.t < P_.t_end) || P_.err || P_.alpha_valid)) continue;
        if (sel == SEL_ACTIVE && (!P_.active || (P_.err & ERR_STAGE_BAD))) continue;
        const int64_t plane = (int64_t)P_.nx * P_.ny;
        const TU* base = U + P_.off_u;
        double mx = 0.0, my = 0.0;
        long long bad = LLONG_MAX;
        // every load of the thread's cells first (lanes past the chunk read
        // its first cell), then the speeds
        constexpr int PER = CHUNK_CELLS / 256;
        double u[PER][K];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = threadIdx.x + 256 * j;
            const int64_t idx = chunk.start + (k < chunk.count ? k : 0);
#pragma unroll
            for (int c = 0; c < K; ++c) u[j][c] = (double)base[c * plane + idx];
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = threadIdx.x + 256 * j;
            if (k < chunk.count) {
                double sx, sy;
                if (wave_speed<FLUX, DIM, K>(u[j], sch, sx, sy)) {
                    mx = fmax(mx, sx);
                    my = fmax(my, sy);
                } else {
                    const int64_t idx = chunk.start + k;
                    if (idx < bad) bad = idx;
                }
            }
        }
        // thread 0 publishes the chunk's maxima; it reads the slots before
        // the reduction (lower bounds of their final values; see publish_max;
        // read at the start, when every block starts at once, they are mostly
        // still zero)
        uint64_t seen_x = 0, seen_y = 0;
        if (threadIdx.x == 0) {
            seen_x = peek_slot(&P_.ax_bits);
            seen_y = peek_slot(&P_.ay_bits);
        }
        mx = wave_max_d(mx);
        my = wave_max_d(my);
        if (__any(bad != LLONG_MAX)) bad = wave_min_ll(bad);
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            smx[wv] = mx;
            smy[wv] = my;
            sbad[wv] = bad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < 4; ++w) {
                mx = fmax(mx, smx[w]);
                my = fmax(my, smy[w]);
                bad = sbad[w] < bad ? sbad[w] : bad;
            }
            // non-negative doubles order like their bit patterns
            publish_max(&P_.ax_bits, mx, seen_x);
            publish_max(&P_.ay_bits, my, seen_y);
            if (bad != LLONG_MAX) {
                atomicMin((long long*)&P_.bad_cell, bad);
                atomicOr(&P_.err, sel == SEL_ACTIVE ? ERR_STAGE_BAD : ERR_STATE_BAD);
            }
        }
        __syncthreads();
    }
}

// dt = min(CFL rule, t_end - t); the CFL rule is cfl*dx^e/alpha_x in 1D and
// cfl/(alpha_x/dx^e + alpha_y/dy^e) in 2D (or the caller's step).  Returns
// whether the problem takes this step.
__device__ __forceinline__ int select_dt(ProbDev& P_, const StepCtl* ctl, int use_dt_in) {
    P_.active = 0;
    P_.last = 0;
    P_.dt = 0.0;
    if (!(P_.t < P_.t_end) || P_.err) return 0;
    double dtc;
    if (use_dt_in) {
        dtc = P_.dt_in;
        if (!(dtc > 0.0)) return 0;
    } else {
        const double ax = as_double(P_.ax_bits), ay = as_double(P_.ay_bits);
        dtc = ctl->dim == 1 ? ctl->cfl * P_.dxe / ax : ctl->cfl / (ax / P_.dxe + ay / P_.dye);
    }
    const double rem = P_.t_end - P_.t;
    const int last = !(dtc < rem);
    P_.dt = last ? rem : dtc;
    P_.last = last;
    P_.active = 1;
    return 1;
}

// own_ctl: the launch is one block that holds every problem and sets the
// step counters itself (no reset kernel before it); otherwise a reset kernel
// has cleared them and the blocks only raise step_active.
__global__ void dt_kernel(ProbDev* probs, StepCtl* ctl, int nprob, int use_dt_in, int own_ctl) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int act = p < nprob ? select_dt(probs[p], ctl, use_dt_in) : 0;
    if (own_ctl) {
        const int any = __syncthreads_or(act);
        if (threadIdx.x == 0) {
            ctl->nactive = 0;
            ctl->step_active = any;
        }
    } else if (act) {
        atomicOr(&ctl->step_active, 1);
    }
}

// t += dt (exactly t_end on the clipped last step); counts problems still
// running and the steps in which anything advanced.
// The speeds stage 3 gathered from the new state become current.
__global__ void finish_kernel(ProbDev* probs, StepCtl* ctl, int nprob) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) {
        ProbDev& P_ = probs[p];
        // a problem whose intermediate stage was not admissible skipped its
        // stages 2 and 3: its state and time stay those of U^n
        if (P_.active && !(P_.err & ERR_STAGE_BAD)) {
            P_.t = P_.last ? P_.t_end : P_.t + P_.dt;
            P_.ax_bits = P_.ax_next;
            P_.ay_bits = P_.ay_next;
            P_.alpha_valid = 1;
        }
        P_.ax_next = 0;
        P_.ay_next = 0;
        if (P_.t < P_.t_end && !P_.err) atomicAdd(&ctl->nactive, 1);
    }
    if (p == 0 && ctl->step_active) ctl->steps += 1;
}

template <class TU, class TD>
__global__ void pack_kernel(int to_internal, double* ext, TU* u, TD* d, int K, int nvar,
                            int64_t ncell) {
    const int64_t n = (int64_t)nvar * K * ncell;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t plane = e / ncell;   // var*K + comp
        const int64_t cell = e - plane * ncell;
        if (plane < K) {
            if (to_internal) u[e] = (TU)ext[e];
            else ext[e] = (double)u[e];
        } else {
            const int64_t de = (plane - K) * ncell + cell;
            if (to_internal) d[de] = (TD)ext[e];
            else ext[e] = (double)d[de];
        }
    }
}

// --------------------------------------------------------------- launchers

hipError_t launch_reset(ProbDev* probs, StepCtl* ctl, int nprob, int sel, hipStream_t s) {
    reset_kernel<<<(nprob + 255) / 256, 256, 0, s>>>(probs, ctl, nprob, sel);
    return hipGetLastError();
}

template <int P>
static hipError_t alpha_dispatch(int flux, int dim, const void* u, ProbDev* probs,
                                 const Chunk* chunks, int nchunks, const Scheme& sch, int sel,
                                 int grid, hipStream_t s) {
    if (dim == 1) {
        if (flux == F_ADV) alpha_kernel<P, F_ADV, 1><<<grid, 256, 0, s>>>(u, probs, chunks, nchunks, sch, sel);
        else if (flux == F_BURGERS) alpha_kernel<P, F_BURGERS, 1><<<grid, 256, 0, s>>>(u, probs, chunks, nchunks, sch, sel);
        else alpha_kernel<P, F_EULER, 1><<<grid, 256, 0, s>>>(u, probs, chunks, nchunks, sch, sel);
    } else {
        if (flux == F_ADV) alpha_kernel<P, F_ADV, 2><<<grid, 256, 0, s>>>(u, probs, chunks, nchunks, sch, sel);
        else if (flux == F_BURGERS) alpha_kernel<P, F_BURGERS, 2><<<grid, 256, 0, s>>>(u, probs, chunks, nchunks, sch, sel);
        else alpha_kernel<P, F_EULER, 2><<<grid, 256, 0, s>>>(u, probs, chunks, nchunks, sch, sel);
    }
    return hipGetLastError();
}

hipError_t launch_alpha(int prec, int flux, int dim, const void* u, ProbDev* probs,
                        const Chunk* chunks, int nchunks, const Scheme& sch, int sel,
                        int grid, hipStream_t s) {
    if (grid <= 0 || grid > nchunks) grid = nchunks;
    if (prec == P_F32) return alpha_dispatch<P_F32>(flux, dim, u, probs, chunks, nchunks, sch, sel, grid, s);
    if (prec == P_KAHAN) return alpha_dispatch<P_KAHAN>(flux, dim, u, probs, chunks, nchunks, sch, sel, grid, s);
    return alpha_dispatch<P_F64>(flux, dim, u, probs, chunks, nchunks, sch, sel, grid, s);
}

hipError_t launch_dt(ProbDev* probs, StepCtl* ctl, int nprob, int use_dt_in, int own_ctl,
                     hipStream_t s) {
    if (own_ctl && nprob > 256) return hipErrorInvalidValue;
    dt_kernel<<<(nprob + 255) / 256, 256, 0, s>>>(probs, ctl, nprob, use_dt_in, own_ctl);
    return hipGetLastError();
}

hipError_t launch_finish(ProbDev* probs, StepCtl* ctl, int nprob, hipStream_t s) {
    finish_kernel<<<(nprob + 255) / 256, 256, 0, s>>>(probs, ctl, nprob);
    return hipGetLastError();
}

hipError_t launch_pack(int prec, int to_internal, double* ext, StateBuf buf, int64_t off_u,
                       int64_t off_d, int K, int nvar, int64_t ncell, hipStream_t s) {
    const int64_t n = (int64_t)nvar * K * ncell;
    const int grid = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (prec == P_F64) {
        pack_kernel<double, double><<<grid, 256, 0, s>>>(to_internal, ext, (double*)buf.u + off_u,
                                                         (double*)buf.d + off_d, K, nvar, ncell);
    } else if (prec == P_F32) {
        pack_kernel<float, float><<<grid, 256, 0, s>>>(to_internal, ext, (float*)buf.u + off_u,
                                                       (float*)buf.d + off_d, K, nvar, ncell);
    } else if (prec == P_ACC64) {
        pack_kernel<double, float><<<grid, 256, 0, s>>>(to_internal, ext, (double*)buf.u + off_u,
                                                        (float*)buf.d + off_d, K, nvar, ncell);
    } else {
        pack_kernel<ffs, float><<<grid, 256, 0, s>>>(to_internal, ext, (ffs*)buf.u + off_u,
                                                     (float*)buf.d + off_d, K, nvar, ncell);
    }
    return hipGetLastError();
}

}  // namespace hweno

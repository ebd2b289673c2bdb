// Fused 1D HWENO stage kernel: reconstruction (Sec. 2.1 Steps 1-3,
// Appendix A; for the Euler equations optionally in local characteristic
// variables, CH), interface values, global Lax-Friedrichs fluxes for f and h,
// the residual of eq. semi-discrete-scheme and the SSP-RK3 stage with the
// modified derivative (Sec. 2.1 Step 4).
//
// A workgroup of 256 threads owns 254 consecutive output cells of one
// problem: it stages the 258 averages and derivative means it needs in LDS
// (coalesced, ghost cells through the boundary index map), reconstructs 256
// cells (one per thread, every component), computes the 255 interface
// fluxes once each, and updates the 254 interior cells.
#pragma once

#include "device_common.h"

namespace hweno {

// Workgroups per CU the register allocation must allow.  With FP32 faces
// the staging in LDS (21.6 KB per workgroup) admits seven; six fit the
// registers of stages 1-3 (stage 3, with the FP64 wave-speed reduction,
// only because it loads its RK inputs late, see stage1d_late_rk); the
// right-hand side and the characteristic projections need more.  With FP64
// faces LDS (37 KB) admits four and the allocation is left to the compiler.
template <int P, int mode, bool CH> constexpr int stage1d_min_blocks() {
    return P == P_F64 ? 1
                      : CH ? (mode == MODE_S3 ? 4 : 5)
                           : (mode == MODE_RHS ? 5 : 6);
}

// Stage 3 of the Euler system in single precision (component-wise) loads
// U^n and the saved derivatives after the reconstruction instead of before
// it: the nine registers they would hold through it are what separates its
// 95 VGPRs (five workgroups per CU) from 80 (six), and the extra workgroup
// hides more latency than the late loads expose.
template <int P, int K, int mode, bool CH> constexpr bool stage1d_late_rk() {
    return mode == MODE_S3 && P != P_F64 && !CH && K > 1;
}

template <int P, int K, int FLUX, int mode, bool CH>
__global__ void __launch_bounds__(256, (stage1d_min_blocks<P, mode, CH>())) stage1d_kernel(StageArgs a) {
    using TU = typename PrecT<P>::TU;
    using TD = typename PrecT<P>::TD;
    using T = typename PrecT<P>::T;
    using TA = typename PrecT<P>::TA;
    constexpr int NL = TILE1D_OUT + 4;   // staged cells
    __shared__ TU su[K][NL];
    __shared__ TD sv[K][NL];
    __shared__ T sR[2 * K][256];         // (u, u_x) at x_{i+1/2} from cell i
    __shared__ T sL[2 * K][256];         // (u, u_x) at x_{i-1/2} from cell i
    // (f-hat, h-hat) at the right interface of cell t: written over sR, whose
    // entry t only thread t reads (right before it writes the flux there)
    T (&sF)[2 * K][256] = sR;
    __shared__ double s_mx[4];           // stage 3: per-wave maxima of the wave speeds
    __shared__ long long s_bad[4];

    const int tid = threadIdx.x;
    const Scheme& sch = a.sch;
    const int squared = sch.weights == W_BETA2;   // W_PAPER prints beta + eps in 1D
    const Flux<T, FLUX, K, 0> F(sch);
    const Tile1D* tiles = (const Tile1D*)a.tiles + a.tile_offset;
    const T g0inv = (T)(1.0 / sch.gam[0]);

    for (int tix = blockIdx.x; tix < a.ntiles; tix += gridDim.x) {
        const Tile1D tile = tiles[tix];
        const ProbDev& P_ = a.probs[tile.prob];
        // stages 2 and 3 skip a problem whose stage input was not admissible
        // (per-stage speeds): its U^n stays as it is
        if (mode != MODE_RHS &&
            (!P_.active || (mode != MODE_S1 && (P_.err & ERR_STAGE_BAD))))
            continue;
        const int nx = P_.nx, bcx = P_.bc_x;
        const T dx = (T)P_.dx, inv_dx = (T)P_.inv_dx;
        const TA inv_dx_a = (TA)P_.inv_dx;
        const T alpha = (T)as_double(P_.ax_bits);
        const double dt = P_.dt;
        const int c0 = tile.c0;
        // problem-table fields are copied before any store: read after one,
        // they would be reloaded (possible aliasing) and waited for
        const int64_t off_u = P_.off_u, off_d = P_.off_d;
        // stage 3: thread 0, which publishes the tile's speed maximum, reads
        // the slot now (a lower bound of its final value; see publish_max)
        uint64_t seen_x = 0;
        if (mode == MODE_S3 && tid == 0) seen_x = peek_slot(&a.probs[tile.prob].ax_next);

        for (int k = tid; k < NL; k += 256) {
            const int src = bc_map(c0 - 2 + k, nx, bcx);
            const bool mir = FLUX == F_EULER && wall_mirrored(c0 - 2 + k, nx, bcx);
#pragma unroll
            for (int c = 0; c < K; ++c) {
                // behind a wall: momentum odd, other averages even, and the
                // derivative means of the opposite parity
                su[c][k] = neg_if(((const TU*)a.in.u)[off_u + (int64_t)c * nx + src], mir && c == 1);
                sv[c][k] = neg_if(((const TD*)a.in.d)[off_d + (int64_t)c * nx + src], mir && c != 1);
            }
        }
        // stages 2 and 3: U^n and the saved derivatives of the output cell
        // (lanes without output read element 0), loaded now so that they
        // arrive while the cell is reconstructed and the fluxes are formed,
        // or after the reconstruction (stage1d_late_rk)
        const int gi = c0 - 1 + tid;
        const bool emit = tid >= 1 && tid <= TILE1D_OUT && gi < nx;
        constexpr bool LATE_RK = stage1d_late_rk<P, K, mode, CH>();
        TA unr[K];
        T hnr[K];
        auto load_rk = [&]() {
            const int gl = emit ? gi : 0;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                unr[c] = (TA)((const TU*)a.un)[off_u + (int64_t)c * nx + gl];
                hnr[c] = (T)((const TD*)a.h)[off_d + (int64_t)c * nx + gl];
            }
        };
        if constexpr ((mode == MODE_S2 || mode == MODE_S3) && !LATE_RK) load_rk();
        __syncthreads();

        // ---- reconstruct local cell tid (global c0 - 1 + tid) ---------------
        // Per field: the differences of the neighbours' averages from the
        // cell's (dm, dp) and dx times their derivative means (dvm, dvp) give
        // the Appendix A quartic (centre average subtracted), the two linear
        // polynomials, the weights, and the combined polynomial's even and
        // odd parts at the faces (E, O) and of its derivative (De, Do).
        auto recon_field = [&](T dm, T dp, T dvm, T dvp, T& E, T& O, T& De, T& Do) {
            T c0v[5];
            c0v[0] = (T)(-47.0 / 480.0) * (dm + dp) + (T)(9.0 / 320.0) * (dvp - dvm);
            c0v[1] = (T)(13.0 / 16.0) * (dp - dm) - (T)(5.0 / 16.0) * (dvm + dvp);
            c0v[2] = (T)(5.0 / 4.0) * (dm + dp) + (T)(3.0 / 8.0) * (dvm - dvp);
            c0v[3] = (T)0.25 * (dm - dp) + (T)0.25 * (dvm + dvp);
            c0v[4] = (T)-0.5 * (dm + dp) + (T)0.25 * (dvp - dvm);
            T beta[3];
            beta[0] = sch.smoothness == BETA_CLASSICAL
                          ? beta_classical_1d(c0v)
                          : c0v[1] * c0v[1] + (T)4 * c0v[2] * c0v[2] + (T)36 * c0v[3] * c0v[3] +
                                (T)576 * c0v[4] * c0v[4];
            beta[1] = dm * dm;
            beta[2] = dp * dp;
            T w[3];
            nonlinear_weights<T, 2, false>(beta, sch, squared, w);
            const T a0 = w[0] * g0inv;
            const T b1 = w[1] - a0 * (T)sch.gam[1], b2 = w[2] - a0 * (T)sch.gam[2];
            T C[5];
#pragma unroll
            for (int l = 0; l < 5; ++l) C[l] = a0 * c0v[l];
            C[1] += b2 * dp - b1 * dm;   // slopes of p1 (-dm) and p2 (dp)
            E = C[0] + (T)0.25 * C[2] + (T)0.0625 * C[4];
            O = (T)0.5 * C[1] + (T)0.125 * C[3];
            De = C[1] + (T)0.75 * C[3];
            Do = C[2] + (T)0.5 * C[4];
        };
        T dm[K], dp[K], dvm[K], dvp[K], E[K], O[K], De[K], Do[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const TU uc = su[c][tid + 1];
            dm[c] = (T)(su[c][tid] - uc);        // u_{i-1} - u_i
            dp[c] = (T)(su[c][tid + 2] - uc);    // u_{i+1} - u_i
            dvm[c] = dx * (T)sv[c][tid];         // dx * v_{i-1}
            dvp[c] = dx * (T)sv[c][tid + 2];     // dx * v_{i+1}
        }
        if constexpr (CH) {
            // local characteristic variables of the cell's own average: the
            // reconstruction is linear in the stencil except for the weights,
            // so the differences project directly and the face values map
            // back with R
            T Uc[K];
#pragma unroll
            for (int c = 0; c < K; ++c) Uc[c] = (T)su[c][tid + 1];
            const Eigen<T, K> ev(Uc, (T)(sch.gas_gamma - 1.0));
            T wm[K], wp[K], wvm[K], wvp[K], e[K], o[K], de[K], dd[K];
            ev.left(dm, wm);
            ev.left(dp, wp);
            ev.left(dvm, wvm);
            ev.left(dvp, wvp);
#pragma unroll
            for (int k = 0; k < K; ++k) recon_field(wm[k], wp[k], wvm[k], wvp[k], e[k], o[k], de[k], dd[k]);
            ev.right(e, E);
            ev.right(o, O);
            ev.right(de, De);
            ev.right(dd, Do);
        } else {
#pragma unroll
            for (int c = 0; c < K; ++c) recon_field(dm[c], dp[c], dvm[c], dvp[c], E[c], O[c], De[c], Do[c]);
        }
        T vhat[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const T ucT = (T)su[c][tid + 1];
            sR[c][tid] = ucT + (E[c] + O[c]);
            sL[c][tid] = ucT + (E[c] - O[c]);
            sR[K + c][tid] = (De[c] + Do[c]) * inv_dx;
            sL[K + c][tid] = (De[c] - Do[c]) * inv_dx;
            vhat[c] = (T)2 * O[c] * inv_dx;   // (u(x+1/2) - u(x-1/2)) / dx
        }
        if constexpr (LATE_RK) load_rk();
        __syncthreads();

        // ---- flux at the interface between local cells tid and tid+1 -------
        if (tid < 255) {
            T UL[K], VL[K], UR[K], VR[K], fL[K], hL[K], fR[K], hR[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                UL[c] = sR[c][tid]; VL[c] = sR[K + c][tid];
                UR[c] = sL[c][tid + 1]; VR[c] = sL[K + c][tid + 1];
            }
            F.side(UL, VL, nullptr, fL, hL, nullptr);
            F.side(UR, VR, nullptr, fR, hR, nullptr);
            const T ha = (T)0.5 * alpha;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                sF[c][tid] = (T)0.5 * (fL[c] + fR[c]) - ha * (UR[c] - UL[c]);
                sF[K + c][tid] = (T)0.5 * (hL[c] + hR[c]) - ha * (VR[c] - VL[c]);
            }
        }
        __syncthreads();

        // ---- residual and RK stage of local cell tid -----------------------
        double unew[K];
        if (emit) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const TA Lu = -((TA)sF[c][tid] - (TA)sF[c][tid - 1]) * inv_dx_a;
                const T Lv = -(sF[K + c][tid] - sF[K + c][tid - 1]) * inv_dx;
                const TA ucur = (TA)su[c][tid + 1];
                const int64_t ou = off_u + (int64_t)c * nx + gi;
                const int64_t od = off_d + (int64_t)c * nx + gi;
                if (mode == MODE_RHS) {
                    const int64_t ob = (int64_t)c * nx + gi;
                    a.L_out[ob] = (double)Lu;
                    a.L_out[(int64_t)K * nx + ob] = (double)Lv;
                    a.Uh_out[ob] = (double)ucur;
                    a.Uh_out[(int64_t)K * nx + ob] = (double)vhat[c];
                } else {
                    TU* Ou = (TU*)a.out.u;
                    TD* Ov = (TD*)a.out.d;
                    const TA dta = (TA)dt;
                    const T dtt = (T)dt;
                    if (mode == MODE_S1) {
                        Ou[ou] = (TU)(ucur + dta * Lu);
                        Ov[od] = (TD)(vhat[c] + dtt * Lv);
                        ((TD*)a.h)[od] = (TD)vhat[c];
                    } else {
                        const T hn = hnr[c];
                        if (mode == MODE_S2) {
                            Ou[ou] = (TU)((TA)0.75 * unr[c] + (TA)0.25 * (ucur + dta * Lu));
                            Ov[od] = (TD)((T)0.75 * hn + (T)0.25 * (vhat[c] + dtt * Lv));
                        } else {
                            const TU nu = (TU)((TA)(1.0 / 3.0) * unr[c] + (TA)(2.0 / 3.0) * (ucur + dta * Lu));
                            Ou[ou] = nu;
                            unew[c] = (double)nu;
                            Ov[od] = (TD)((T)(1.0 / 3.0) * hn + (T)(2.0 / 3.0) * (vhat[c] + dtt * Lv));
                        }
                    }
                }
            }
        }
        if (mode == MODE_S3) {
            // largest x wave speed of the state being written (the 1D time
            // step uses no other), for the next step: reduced over the wave
            // here and over the workgroup below; the first non-admissible
            // cell is reduced only where there is one
            double mx = 0.0;
            long long bad = LLONG_MAX;
            if (emit) {
                double sx, sy;
                if (wave_speed<FLUX, 1, K>(unew, sch, sx, sy)) mx = sx;
                else bad = gi;
            }
            mx = wave_max_d(mx);
            if (__any(bad != LLONG_MAX)) bad = wave_min_ll(bad);
            if ((tid & 63) == 0) {
                s_mx[tid >> 6] = mx;
                s_bad[tid >> 6] = bad;
            }
        }
        __syncthreads();   // LDS reuse by the next tile
        if (mode == MODE_S3 && tid == 0) {
            double mx = s_mx[0];
            long long bad = s_bad[0];
#pragma unroll
            for (int w = 1; w < 4; ++w) {
                mx = fmax(mx, s_mx[w]);
                bad = s_bad[w] < bad ? s_bad[w] : bad;
            }
            publish_reduced(a.probs[tile.prob], mx, 0.0, bad, seen_x, 0);
        }
    }
}

}  // namespace hweno

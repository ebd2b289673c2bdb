// 2D Euler stage kernel with the HWENO reconstruction and derivative
// modification in local characteristic variables (remark closing Sec. 2.2):
// each cell's stencil is projected with the eigenvectors of the flux
// Jacobian at the cell's own average, once with those of F (x) and once with
// those of G (y); every characteristic field is reconstructed as a scalar
// (Sec. 2.2 Steps 1-3, Appendix A), the x-edge values and v-hat come from the
// x-projected polynomials and the y-edge values and w-hat from the
// y-projected ones, and are mapped back to conserved variables with R.
// Fluxes, residual and RK stage are those of the component-wise kernel.
//
// Work decomposition as in stage2d_kernel (64-column strip, rows marched
// upwards, wave k = characteristic field k, lane = column), with one change:
// a projection mixes all four components of every stencil entry, so the
// rows of the march live in an LDS ring of four rows (all components) that
// every wave reads, instead of per-wave registers.  Per row r:
//   top  each wave writes its component of row r+2 (loaded one row earlier)
//        into the ring slot of row r-2, which nothing reads any more;
//   R    wave k projects the stencil of its lane's cell with row k of L_x
//        and of L_y, reconstructs both fields and writes the face values as
//        characteristic differences from the cell average to LDS;
//   F    each wave maps the hats of its own lane back (row c of R, kept from
//        R); each thread forms the conserved values on both sides of one
//        edge point from the characteristic differences, the two cells'
//        averages and their R, and the Lax-Friedrichs flux;
//   S    residual and RK stage of row r-1, as in the component-wise kernel.
#pragma once

#include "stage2d.h"

namespace hweno {

template <int P, int Q, int mode>
__global__ void __launch_bounds__(256, (P == P_F64 ? 1 : 2)) stage2d_char_kernel(StageArgs a) {
    constexpr int K = 4;
    using TU = typename PrecT<P>::TU;
    using TD = typename PrecT<P>::TD;
    using T = typename PrecT<P>::T;
    using TA = typename PrecT<P>::TA;
    constexpr int NF = Q * 3 * K;
    // characteristic differences at the Gauss points of the faces
    __shared__ T sxR[NF][64], sxL[NF][64], syB[NF][64], syT[NF][64];
    __shared__ T sFX[Q][3 * K][64], sFY[Q][3 * K][64];
    __shared__ TU rU[4][K][64];          // ring of rows: cell averages
    __shared__ TD rV[4][K][64], rW[4][K][64];   // and derivative averages
    __shared__ T sHc[2][K][64];          // characteristic hats of the row
    __shared__ double snew[2][K][64];    // stage 3: new averages of two output rows
    __shared__ double smx[64], smy[64];
    __shared__ long long sbad[64];

    const int lane = threadIdx.x & 63;
    const int c = threadIdx.x >> 6;   // component of this wave's loads; field of its reconstruction
    const Scheme& sch = a.sch;
    const int squared = sch.weights == W_BETA2 || (sch.weights == W_PAPER);
    const Flux<T, F_EULER, K, 0> FXf(sch);
    const Flux<T, F_EULER, K, 1> FYf(sch);
    const T gm1 = (T)(sch.gas_gamma - 1.0);
    const Tile2D* tiles = (const Tile2D*)a.tiles + a.tile_offset;
    // y-direction component order (rho, m_y, m_x, E) -> storage index
    constexpr int PY[4] = {0, 2, 1, 3};

    constexpr bool fuse_alpha = mode == MODE_S3;
    if (fuse_alpha && c == 0) {   // ordered before the first gather by a barrier
        smx[lane] = 0.0;
        smy[lane] = 0.0;
        sbad[lane] = LLONG_MAX;
    }

    for (int tix = blockIdx.x; tix < a.ntiles; tix += gridDim.x) {
        const Tile2D tile = tiles[tix];
        const ProbDev& P_ = a.probs[tile.prob];
        // stages 2 and 3 skip a problem whose stage input was not admissible
        // (per-stage speeds): its U^n stays as it is
        if (mode != MODE_RHS &&
            (!P_.active || (mode != MODE_S1 && (P_.err & ERR_STAGE_BAD))))
            continue;
        const int nx = P_.nx, ny = P_.ny, bcx = P_.bc_x, bcy = P_.bc_y;
        const int64_t plane = (int64_t)nx * ny;
        const T inv_dx = (T)P_.inv_dx, inv_dy = (T)P_.inv_dy;
        const TA inv_dx_a = (TA)P_.inv_dx, inv_dy_a = (TA)P_.inv_dy;
        const T rx = (T)(P_.dx * P_.inv_dy), ry = (T)(P_.dy * P_.inv_dx);
        const T ax = (T)as_double(P_.ax_bits), ay = (T)as_double(P_.ay_bits);
        const double dt = P_.dt;
        const int gi = tile.i0 - 2 + lane;
        const int li = bc_map(gi, nx, bcx);
        const bool out_col = lane >= 2 && lane < 62 && gi < nx;
        const int64_t off_u = P_.off_u, off_d = P_.off_d;
        const TU* Uu = (const TU*)a.in.u + off_u + c * plane;
        const TD* Uv = (const TD*)a.in.d + off_d + c * plane;
        const TD* Uw = (const TD*)a.in.d + off_d + (K + c) * plane;
        const TU* Un = (const TU*)a.un + off_u + c * plane;
        TD* Hv = (TD*)a.h + off_d + c * plane;
        TD* Hw = (TD*)a.h + off_d + (K + c) * plane;
        TU* Ou = (TU*)a.out.u + off_u + c * plane;
        TD* Ov = (TD*)a.out.d + off_d + c * plane;
        TD* Ow = (TD*)a.out.d + off_d + (K + c) * plane;

        const bool mx = wall_mirrored(gi, nx, bcx);
        const bool nux = mx && c == 1, nvx = mx && c != 1, nwx = mx && c == 1;
        auto load_row = [&](int j, TU& u, TD& v, TD& w) {
            const int64_t o = (int64_t)bc_map(j, ny, bcy) * nx + li;
            const bool my = wall_mirrored(j, ny, bcy);
            const bool nuy = my && c == 2, nvy = my && c == 2, nwy = my && c != 2;
            u = neg_if(Uu[o], nux != nuy);
            v = neg_if(Uv[o], nvx != nvy);
            w = neg_if(Uw[o], nwx != nwy);
        };
        auto put_row = [&](int j, TU u, TD v, TD w) {
            rU[j & 3][c][lane] = u;
            rV[j & 3][c][lane] = v;
            rW[j & 3][c][lane] = w;
        };
        const int j0 = tile.j0, jend = tile.j0 + tile.nrows;

        // row `row`'s speeds are gathered by wave w (rotating with the row in
        // the march, so that the gathers spread over the SIMDs; per-lane
        // maxima in LDS, cleared by the wave that publishes them)
        auto gather_wave = [](int row) { return (int)((unsigned)row % (unsigned)K); };
        auto gather_speeds = [&](int row, int w) {
            if (c == w && out_col) {
                double u[K];
#pragma unroll
                for (int k = 0; k < K; ++k) u[k] = snew[row & 1][k][lane];
                double sx, sy;
                if (wave_speed<F_EULER, 2, K>(u, sch, sx, sy)) {
                    smx[lane] = fmax(smx[lane], sx);
                    smy[lane] = fmax(smy[lane], sy);
                } else {
                    const long long idx = (long long)row * nx + gi;
                    if (idx < sbad[lane]) sbad[lane] = idx;
                }
            }
        };

        // prologue: rows j0-2 .. j0 into the ring, row j0+1 prefetched
        TU um, u0, up, un_;
        TD vn_, wn_;
        {
            TD v, w;
            load_row(j0 - 2, um, v, w);
            put_row(j0 - 2, um, v, w);
            load_row(j0 - 1, u0, v, w);
            put_row(j0 - 1, u0, v, w);
            load_row(j0, up, v, w);
            put_row(j0, up, v, w);
        }
        load_row(j0 + 1, un_, vn_, wn_);
        __syncthreads();

        T ytop[Q][3];
        // previous row's flux sums: x differences and y sums of the
        // cell-average fluxes in the accumulation type, of the derivative
        // fluxes in T
        TA xdu_prev = 0, gyu_prev = 0;
        T xdd_prev[2] = {0, 0}, gyd_prev[2] = {0, 0};
        T hat_prev[2] = {0, 0};
        const int lm = lane > 0 ? lane - 1 : 0, lp = lane < 63 ? lane + 1 : 63;

        for (int r = j0 - 1; r <= jend; ++r) {
            if (fuse_alpha && r - 3 >= j0) gather_speeds(r - 3, gather_wave(r - 3));
            // ring: row r+2 into the slot of row r-2; prefetch row r+3
            const TU u2 = un_;
            put_row(r + 2, un_, vn_, wn_);
            load_row(r + 3, un_, vn_, wn_);

            TA unr = 0;
            T hvr = 0, hwr = 0;
            const bool emit = r > j0 && out_col;
            const int64_t oo = (int64_t)(r - 1) * nx + gi;
            if (mode == MODE_S2 || mode == MODE_S3) {
                const int64_t ol = emit ? oo : 0;
                unr = (TA)Un[ol];
                hvr = (T)Hv[ol];
                hwr = (T)Hw[ol];
            }

            // ---- R: field c of the cell (gi, r), in x and y projections ----
            if (r > j0 - 1) {
#pragma unroll
                for (int mu = 0; mu < Q; ++mu)
#pragma unroll
                    for (int v = 0; v < 3; ++v) syT[(mu * 3 + v) * K + c][lane] = ytop[mu][v];
            }
            const int sm = (r - 1) & 3, s0 = r & 3, sp = (r + 1) & 3;
            T Rx[K], Ry[K];   // row c of R_x, row of R_y giving component c
            T wx[17], wy[17];
            {
                T Uc[K], Uy[K];
#pragma unroll
                for (int k = 0; k < K; ++k) Uc[k] = (T)rU[s0][k][lane];
#pragma unroll
                for (int k = 0; k < K; ++k) Uy[k] = Uc[PY[k]];
                const Eigen<T, K> ex(Uc, gm1);
                const Eigen<T, K> ey(Uy, gm1);
                // row c of R_x; row PY[c] of R_y (component c in y order); row
                // c of L_x and of L_y (field c)
                const int cy = c == 1 ? 2 : (c == 2 ? 1 : c);
                T Lx[K], Ly[K];
                ex.rrow(c, Rx);
                ey.rrow(cy, Ry);
                ex.lrow(c, Lx);
                ey.lrow(c, Ly);
#pragma unroll
                for (int e = 0; e < 17; ++e) {
                    wx[e] = 0;
                    wy[e] = 0;
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const TU uc = rU[s0][k][lane];
                    T q[17];
                    q[0] = (T)(rU[sm][k][lm] - uc);
                    q[1] = (T)(rU[sm][k][lane] - uc);
                    q[2] = (T)(rU[sm][k][lp] - uc);
                    q[3] = (T)(rU[s0][k][lm] - uc);
                    q[4] = (T)0;
                    q[5] = (T)(rU[s0][k][lp] - uc);
                    q[6] = (T)(rU[sp][k][lm] - uc);
                    q[7] = (T)(rU[sp][k][lane] - uc);
                    q[8] = (T)(rU[sp][k][lp] - uc);
                    q[9] = (T)rV[s0][k][lm];
                    q[10] = (T)rV[s0][k][lp];
                    q[11] = (T)rV[sm][k][lane];
                    q[12] = (T)rV[sp][k][lane];
                    q[13] = (T)rW[s0][k][lm];
                    q[14] = (T)rW[s0][k][lp];
                    q[15] = (T)rW[sm][k][lane];
                    q[16] = (T)rW[sp][k][lane];
                    // storage component k is position k of the x order and
                    // position PY[k] of the y order
                    const T lx = Lx[k], ly = Ly[PY[k]];
#pragma unroll
                    for (int e = 0; e < 17; ++e) {
                        wx[e] += lx * q[e];
                        wy[e] += ly * q[e];
                    }
                }
            }
            T vhx, why;
            {
                T C[15], vh, wh;
                reconstruct2d<T>(wx, sch, squared, C, vh, wh);
                vhx = vh;
                // derivatives in local units (d/dxi, d/deta): the back
                // projection and the edge flux are linear in them, and the
                // residual applies 1/dx, 1/dy once
                T val[2][Q], dn[2][Q], dtg[2][Q];
                face_values<T, Q>(C, val, dn, dtg);
#pragma unroll
                for (int mu = 0; mu < Q; ++mu) {
                    sxL[(mu * 3 + 0) * K + c][lane] = val[0][mu];
                    sxL[(mu * 3 + 1) * K + c][lane] = dn[0][mu];
                    sxL[(mu * 3 + 2) * K + c][lane] = dtg[0][mu];
                    sxR[(mu * 3 + 0) * K + c][lane] = val[1][mu];
                    sxR[(mu * 3 + 1) * K + c][lane] = dn[1][mu];
                    sxR[(mu * 3 + 2) * K + c][lane] = dtg[1][mu];
                }
            }
            {
                T C[15], vh, wh;
                reconstruct2d<T>(wy, sch, squared, C, vh, wh);
                why = wh;
                T D[15];
                transpose15(C, D);
                T val[2][Q], dn[2][Q], dtg[2][Q];
                face_values<T, Q>(D, val, dn, dtg);
#pragma unroll
                for (int mu = 0; mu < Q; ++mu) {
                    syB[(mu * 3 + 0) * K + c][lane] = val[0][mu];
                    syB[(mu * 3 + 1) * K + c][lane] = dtg[0][mu];
                    syB[(mu * 3 + 2) * K + c][lane] = dn[0][mu];
                    ytop[mu][0] = val[1][mu];
                    ytop[mu][1] = dtg[1][mu];
                    ytop[mu][2] = dn[1][mu];
                }
            }
            sHc[0][c][lane] = vhx;
            sHc[1][c][lane] = why;

            T hat[2];
            if (r > j0 - 1) {
                __syncthreads();  // A: face values of row r (and top faces of r-1) ready
                // ---- hats of this lane's cell, component c ------------------
                {
                    T hv = 0, hw = 0;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        hv += Rx[k] * sHc[0][k][lane];
                        hw += Ry[k] * sHc[1][k][lane];
                    }
                    hat[0] = hv;
                    hat[1] = hw;
                }
                // ---- F: edge fluxes ---------------------------------------
                for (int sl = threadIdx.x; sl < 2 * Q * 64; sl += 64 * K) {
                    const int kind = sl / (Q * 64);
                    const int mu = (sl >> 6) % Q;
                    const int l = sl & 63;
                    T UL[K], VL[K], WL[K], UR[K], VR[K], WR[K], out[3 * K];
                    // conserved values on one side: average + R (differences)
                    auto side = [&](int slot, int cl, int dir, const T (*src)[64], T* U, T* V,
                                    T* W) {
                        T Uc[K], Ud[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) Uc[k] = (T)rU[slot][k][cl];
#pragma unroll
                        for (int k = 0; k < K; ++k) Ud[k] = dir ? Uc[PY[k]] : Uc[k];
                        const Eigen<T, K> ev(Ud, gm1);
                        T du[K], dv[K], dw[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            du[k] = src[(mu * 3 + 0) * K + k][cl];
                            dv[k] = src[(mu * 3 + 1) * K + k][cl];
                            dw[k] = src[(mu * 3 + 2) * K + k][cl];
                        }
                        T pu[K], pv[K], pw[K];
                        ev.right(du, pu);
                        ev.right(dv, pv);
                        ev.right(dw, pw);
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const int s = dir ? PY[k] : k;
                            U[s] = Uc[s] + pu[k];
                            V[s] = pv[k];
                            W[s] = pw[k];
                        }
                    };
                    if (kind == 0) {
                        if (l < 63) {   // x-edge between lanes l and l+1 of row r
                            side(s0, l, 0, sxR, UL, VL, WL);
                            side(s0, l + 1, 0, sxL, UR, VR, WR);
                            lf_edge<T, F_EULER, K, 0>(FXf, UL, VL, WL, UR, VR, WR, ax, out);
#pragma unroll
                            for (int k = 0; k < 3 * K; ++k) sFX[mu][k][l] = out[k];
                        }
                    } else {            // y-edge between rows r-1 and r, column l
                        side(sm, l, 1, syT, UL, VL, WL);
                        side(s0, l, 1, syB, UR, VR, WR);
                        lf_edge<T, F_EULER, K, 1>(FYf, UL, VL, WL, UR, VR, WR, ay, out);
#pragma unroll
                        for (int k = 0; k < 3 * K; ++k) sFY[mu][k][l] = out[k];
                    }
                }
                __syncthreads();  // B: fluxes ready
                // ---- S: residual and RK stage of row r-1 ------------------
                // The derivative fluxes are differenced in T: the difference of
                // two T values rounded to T is what a wider difference rounds to.
                TA xdu = 0, gyu = 0;
                T xdd[2], gyd[2];
#pragma unroll
                for (int sk = 0; sk < 3; ++sk) {
                    T fr = 0, fl = 0, g = 0;
#pragma unroll
                    for (int mu = 0; mu < Q; ++mu) {
                        const T w = (T)(0.5 * Gauss<Q>::w(mu));   // fluxes are stored doubled
                        fr += w * sFX[mu][sk * K + c][lane];
                        fl += w * sFX[mu][sk * K + c][lane > 0 ? lane - 1 : 0];
                        g += w * sFY[mu][sk * K + c][lane];
                    }
                    if (sk == 0) {
                        xdu = (TA)fr - (TA)fl;
                        gyu = (TA)g;
                    } else {
                        xdd[sk - 1] = fr - fl;
                        gyd[sk - 1] = g;
                    }
                }
                if (r > j0) {
                    const TA Lu = -(xdu_prev * inv_dx_a + (gyu - gyu_prev) * inv_dy_a);
                    // v- and w-fluxes carry the derivatives in local units
                    const T Lv = -inv_dx * (xdd_prev[0] + rx * (gyd[0] - gyd_prev[0]));
                    const T Lw = -inv_dy * (ry * xdd_prev[1] + (gyd[1] - gyd_prev[1]));
                    if (emit) {
                        const TA ucur = (TA)um;   // u-bar of row r-1 in the input set
                        if (mode == MODE_RHS) {
                            const int64_t ob = (int64_t)c * plane + oo;
                            a.L_out[ob] = (double)Lu;
                            a.L_out[K * plane + ob] = (double)Lv;
                            a.L_out[2 * K * plane + ob] = (double)Lw;
                            a.Uh_out[ob] = (double)ucur;
                            a.Uh_out[K * plane + ob] = (double)hat_prev[0];
                            a.Uh_out[2 * K * plane + ob] = (double)hat_prev[1];
                        } else {
                            const TA dta = (TA)dt;
                            const T dtt = (T)dt;
                            if (mode == MODE_S1) {
                                Ou[oo] = (TU)(ucur + dta * Lu);
                                Ov[oo] = (TD)(hat_prev[0] + dtt * Lv);
                                Ow[oo] = (TD)(hat_prev[1] + dtt * Lw);
                                Hv[oo] = (TD)hat_prev[0];
                                Hw[oo] = (TD)hat_prev[1];
                            } else if (mode == MODE_S2) {
                                Ou[oo] = (TU)((TA)0.75 * unr + (TA)0.25 * (ucur + dta * Lu));
                                Ov[oo] = (TD)((T)0.75 * hvr + (T)0.25 * (hat_prev[0] + dtt * Lv));
                                Ow[oo] = (TD)((T)0.75 * hwr + (T)0.25 * (hat_prev[1] + dtt * Lw));
                            } else {
                                const TA third = (TA)(1.0 / 3.0), two3 = (TA)(2.0 / 3.0);
                                const TU nu = (TU)(third * unr + two3 * (ucur + dta * Lu));
                                Ou[oo] = nu;
                                snew[(r - 1) & 1][c][lane] = (double)nu;
                                Ov[oo] = (TD)((T)(1.0 / 3.0) * hvr +
                                              (T)(2.0 / 3.0) * (hat_prev[0] + dtt * Lv));
                                Ow[oo] = (TD)((T)(1.0 / 3.0) * hwr +
                                              (T)(2.0 / 3.0) * (hat_prev[1] + dtt * Lw));
                            }
                        }
                    }
                }
                xdu_prev = xdu;
                gyu_prev = gyu;
#pragma unroll
                for (int sk = 0; sk < 2; ++sk) {
                    xdd_prev[sk] = xdd[sk];
                    gyd_prev[sk] = gyd[sk];
                }
            } else {
                // first row (j0-1): no edge of an output row yet; its hats are
                // never used
                hat[0] = hat[1] = 0;
                __syncthreads();   // the ring slot written above is read next row
            }
            hat_prev[0] = hat[0];
            hat_prev[1] = hat[1];
            um = u0; u0 = up; up = u2;
        }
        __syncthreads();  // LDS reuse by the next tile
        if (fuse_alpha) {
            // the last two rows by one wave: no barrier between them
            const int pw = gather_wave(jend - 1);
            if (jend - 2 >= j0) gather_speeds(jend - 2, pw);
            gather_speeds(jend - 1, pw);
            if (c == pw) {
                ProbDev& Pw = a.probs[tile.prob];
                const uint64_t seen_x = peek_slot(&Pw.ax_next), seen_y = peek_slot(&Pw.ay_next);
                const double mxl = smx[lane], myl = smy[lane];
                const long long badl = sbad[lane];
                smx[lane] = 0.0;
                smy[lane] = 0.0;
                sbad[lane] = LLONG_MAX;
                publish_next_speeds(Pw, mxl, myl, badl, seen_x, seen_y);
            }
        }
    }
}

}  // namespace hweno

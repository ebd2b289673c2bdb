// Fused 2D HWENO stage kernel: reconstruction (Sec. 2.2 Steps 1-3,
// Appendix A), Gauss-point edge values, global Lax-Friedrichs edge fluxes,
// the residual of eq. 2D-semi-discrete-scheme-uniform and the SSP-RK3 stage
// combination with the modified derivatives (Sec. 2.2 Step 4), in one pass.
//
// Work decomposition ("column march"): a workgroup owns a strip of 64
// consecutive columns (60 output columns plus two halo columns per side) and
// marches up through a segment of rows.  Wave c handles conserved component
// c, one column per lane, so the x-neighbours of the stencil come from the
// adjacent lanes and the rows below/above stay in registers as the march
// advances.  Per row:
//   R  each (lane, component) reconstructs its cell and writes the values of
//      U, u_xi, u_eta (local units) at the Gauss points of its four faces to
//      LDS;
//   F  each thread computes the Lax-Friedrichs flux (all components) at one
//      edge Gauss point: the x-edges of this row and the y-edges between this
//      row and the one below;
//   S  each (lane, component) differences the fluxes of the row below, which
//      now has all four edges, and applies the RK stage to it.
// Every edge flux is computed once per workgroup and used by both cells, so
// the update is conservative to the rounding of the cell-average arithmetic.
#pragma once

#include "device_common.h"

namespace hweno {

// Gauss-Legendre nodes on [-1/2, 1/2] (ascending) and weights summing to one.
template <int Q> struct Gauss;
template <> struct Gauss<2> {
    static constexpr double g = 0.28867513459481288225;  // 1 / (2 sqrt 3)
    __device__ static constexpr double w(int) { return 0.5; }
};
template <> struct Gauss<3> {
    static constexpr double g = 0.38729833462074168852;  // sqrt(15) / 10
    __device__ static constexpr double w(int mu) { return mu == 1 ? 8.0 / 18.0 : 5.0 / 18.0; }
};

// Appendix A coefficients c_{0,1..15} (stored 0..14) of the quartic p0 in
// terms of q_1..q_17, written with the centre average subtracted from the
// nine averages (q_5 = 0): every coefficient but the constant is invariant
// under that shift, and the constant becomes relative to the centre.
template <class T>
__device__ __forceinline__ void appendix_a(const T* q, T* c) {
    // q[0..16] hold q_1..q_17
    const T q1 = q[0], q2 = q[1], q3 = q[2], q4 = q[3], q6 = q[5], q7 = q[6], q8 = q[7],
            q9 = q[8];
    const T corner = (q1 + q3) + (q7 + q9);
    const T xdc = (q3 + q9) - (q1 + q7);
    const T ydc = (q7 + q9) - (q1 + q3);
    const T xyc = (q1 - q3) - (q7 - q9);
    const T sx = q4 + q6, dxs = q6 - q4;
    const T sy = q2 + q8, dys = q8 - q2;
    const T vWEs = q[9] + q[10], vWEd = q[10] - q[9];
    const T vSNs = q[11] + q[12], vSNd = q[12] - q[11];
    const T wWEs = q[13] + q[14], wWEd = q[14] - q[13];
    const T wSNs = q[15] + q[16], wSNd = q[16] - q[15];
    c[0] = ((T)5 * corner - (T)292 * (sx + sy) + (T)81 * (vWEd + wSNd)) * (T)(1.0 / 2880.0);
    c[1] = ((T)19 * dxs - (T)2 * xdc - (T)6 * vWEs + (T)3 * vSNs) * (T)(1.0 / 24.0);
    c[2] = ((T)19 * dys - (T)2 * ydc + (T)3 * wWEs - (T)6 * wSNs) * (T)(1.0 / 24.0);
    c[3] = ((T)62 * sx + (T)2 * sy - corner - (T)18 * vWEd) * (T)(1.0 / 48.0);
    c[4] = ((T)5 * (vSNd + wWEd) - (T)3 * xyc) * (T)0.125;
    c[5] = ((T)62 * sy + (T)2 * sx - corner - (T)18 * wSNd) * (T)(1.0 / 48.0);
    c[6] = (xdc - (T)4 * dxs + (T)4 * vWEs - (T)2 * vSNs) * (T)0.05;
    c[7] = (ydc - (T)2 * dys) * (T)0.25;
    c[8] = (xdc - (T)2 * dxs) * (T)0.25;
    c[9] = (ydc - (T)4 * dys - (T)2 * wWEs + (T)4 * wSNs) * (T)0.05;
    c[10] = (vWEd - (T)2 * sx) * (T)0.25;
    c[11] = (xyc - (T)2 * vSNd) * (T)0.25;
    c[12] = (corner - (T)2 * (sx + sy)) * (T)0.25;
    c[13] = (xyc - (T)2 * wWEd) * (T)0.25;
    c[14] = (wSNd - (T)2 * sy) * (T)0.25;
}

// HWENO polynomial of one cell and component (Steps 1-3).  q: stencil with
// the centre average subtracted.  C: coefficients of u_ij - u-bar_ij in the
// basis 1, xi, eta, xi^2, xi eta, eta^2, xi^3, xi^2 eta, xi eta^2, eta^3,
// xi^4, xi^3 eta, xi^2 eta^2, xi eta^3, eta^4.
template <class T>
__device__ __forceinline__ void reconstruct2d(const T* q, const Scheme& s, int squared, T* C,
                                              T& vhat, T& what) {
    T c0[15];
    appendix_a(q, c0);
    // linear polynomials on the L-shaped stencils S1..S4: slopes only
    const T sW = -q[3], sE = q[5], sS = -q[1], sN = q[7];
    // smoothness indicators: sum over monomials of (m! n! c_mn)^2
    T b0 = c0[1] * c0[1] + c0[2] * c0[2] + c0[4] * c0[4];
    b0 += (T)4 * (c0[3] * c0[3] + c0[5] * c0[5] + c0[7] * c0[7] + c0[8] * c0[8]);
    b0 += (T)16 * c0[12] * c0[12];
    b0 += (T)36 * (c0[6] * c0[6] + c0[9] * c0[9] + c0[11] * c0[11] + c0[13] * c0[13]);
    b0 += (T)576 * (c0[10] * c0[10] + c0[14] * c0[14]);
    T beta[5];
    beta[0] = s.smoothness == BETA_CLASSICAL ? beta_classical_2d(c0) : b0;
    const T sW2 = sW * sW, sE2 = sE * sE, sS2 = sS * sS, sN2 = sN * sN;
    beta[1] = sW2 + sS2;
    beta[2] = sE2 + sS2;
    beta[3] = sE2 + sN2;
    beta[4] = sW2 + sN2;
    T w[5];
    nonlinear_weights<T, 4, true>(beta, s, squared, w);
    // u_ij = w0/g0 p0 + sum_m (w_m - w0 g_m/g0) p_m   (eq. hweno-reconstruction-2D)
    const T a0 = w[0] * (T)(1.0 / s.gam[0]);
    T bm[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) bm[m] = w[m + 1] - a0 * (T)s.gam[m + 1];
#pragma unroll
    for (int l = 0; l < 15; ++l) C[l] = a0 * c0[l];
    C[1] += sW * (bm[0] + bm[3]) + sE * (bm[1] + bm[2]);
    C[2] += sS * (bm[0] + bm[1]) + sN * (bm[2] + bm[3]);
    // modified derivatives: integrals of u_x, u_y over the cell (scaled units)
    vhat = C[1] + (T)0.25 * C[6] + (T)(1.0 / 12.0) * C[8];
    what = C[2] + (T)0.25 * C[9] + (T)(1.0 / 12.0) * C[7];
}

// Values at the Gauss points of the two faces normal to the first variable
// of C (xi for x-faces; pass the transposed coefficients for y-faces).
// Outputs per side s (0: -1/2, 1: +1/2) and node mu: value, derivative
// normal to the face, derivative along the face (local units, relative
// value).
template <class T, int Q>
__device__ __forceinline__ void face_values(const T* C, T (*val)[Q], T (*dn)[Q], T (*dt)[Q]) {
    const T E0 = C[0] + (T)0.25 * C[3] + (T)0.0625 * C[10], O0 = (T)0.5 * C[1] + (T)0.125 * C[6];
    const T E1 = C[2] + (T)0.25 * C[7], O1 = (T)0.5 * C[4] + (T)0.125 * C[11];
    const T E2 = C[5] + (T)0.25 * C[12], O2 = (T)0.5 * C[8];
    const T E3 = C[9], O3 = (T)0.5 * C[13];
    const T E4 = C[14];
    const T Eb0 = C[1] + (T)0.75 * C[6], Ob0 = C[3] + (T)0.5 * C[10];
    const T Eb1 = C[4] + (T)0.75 * C[11], Ob1 = C[7];
    const T Eb2 = C[8], Ob2 = C[12];
    const T Eb3 = C[13];
    const T g = (T)Gauss<Q>::g, g2 = g * g, g3 = g2 * g, g4 = g2 * g2;
    // symmetric pair of nodes +-g
    const T uee = E0 + g2 * E2 + g4 * E4, uoe = O0 + g2 * O2;
    const T ueo = g * E1 + g3 * E3, uoo = g * O1 + g3 * O3;
    const T nee = Eb0 + g2 * Eb2, noe = Ob0 + g2 * Ob2;
    const T neo = g * Eb1 + g3 * Eb3, noo = g * Ob1;
    const T tee = E1 + (T)3 * g2 * E3, toe = O1 + (T)3 * g2 * O3;
    const T teo = (T)2 * g * E2 + (T)4 * g3 * E4, too = (T)2 * g * O2;
    constexpr int lo = 0, hi = Q - 1;  // nodes -g and +g
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T sg = s ? (T)1 : (T)-1;
        const T ue = uee + sg * uoe, uo = ueo + sg * uoo;
        const T ne = nee + sg * noe, no = neo + sg * noo;
        const T te = tee + sg * toe, to = teo + sg * too;
        val[s][lo] = ue - uo; val[s][hi] = ue + uo;
        dn[s][lo] = ne - no;  dn[s][hi] = ne + no;
        dt[s][lo] = te - to;  dt[s][hi] = te + to;
        if (Q == 3) {
            val[s][1] = E0 + sg * O0;
            dn[s][1] = Eb0 + sg * Ob0;
            dt[s][1] = E1 + sg * O1;
        }
    }
}

template <class T> __device__ __forceinline__ void transpose15(const T* C, T* D) {
    D[0] = C[0]; D[1] = C[2]; D[2] = C[1]; D[3] = C[5]; D[4] = C[4]; D[5] = C[3];
    D[6] = C[9]; D[7] = C[8]; D[8] = C[7]; D[9] = C[6]; D[10] = C[14]; D[11] = C[13];
    D[12] = C[12]; D[13] = C[11]; D[14] = C[10];
}

// Lax-Friedrichs flux at one edge point, all components, TWICE its value:
// out = 2 (f, f^v, f^w) = (f(L) + alpha L) + (f(R) - alpha R).  The factor
// 1/2 is folded into the Gauss weights of the residual, which saves one
// multiply per output (halving and doubling are exact in binary floating
// point); the two sides are accumulated one after the other, so that only
// one side's values and fluxes are live at a time.
template <class T, int FLUX, int K, int DIR>
__device__ __forceinline__ void lf_edge(const Flux<T, FLUX, K, DIR>& F, const T* UL, const T* VL,
                                        const T* WL, const T* UR, const T* VR, const T* WR,
                                        T alpha, T* out) {
    T f[K], fv[K], fw[K];
    F.side(UL, VL, WL, f, fv, fw);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        out[c] = f[c] + alpha * UL[c];
        out[K + c] = fv[c] + alpha * VL[c];
        out[2 * K + c] = fw[c] + alpha * WL[c];
    }
    F.side(UR, VR, WR, f, fv, fw);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        out[c] = (out[c] + f[c]) - alpha * UR[c];
        out[K + c] = (out[K + c] + fv[c]) - alpha * VR[c];
        out[2 * K + c] = (out[2 * K + c] + fw[c]) - alpha * WR[c];
    }
}

// Workgroups per CU the register allocation is made for (launch bounds).
// Variant 0: the occupancy the face arrays and registers comfortably allow
// (every stage fits four FP32-face workgroups in 128 registers, the edge
// flux accumulating one side at a time and stage 3's speed gather being a
// call of its own after the march; with FP64 faces the streamed edge flux
// keeps every stage within the 168 registers of three workgroups, which
// their 48 KB of LDS also allow); variant 1: one workgroup more per CU,
// which caps the registers lower (the compiler may spill).  The tuner picks.
template <int P, int Q, int mode, int V> constexpr int stage2d_min_blocks() {
    return V + (P == P_F64 ? (Q == 3 ? 1 : 2) : (Q == 3 ? 2 : 4));
}

template <int P, int K, int Q, int FLUX, int mode, int V>
__global__ void __launch_bounds__(64 * K, (stage2d_min_blocks<P, Q, mode, V>())) stage2d_kernel(StageArgs a) {
    using TU = typename PrecT<P>::TU;
    using TD = typename PrecT<P>::TD;
    using T = typename PrecT<P>::T;
    using TA = typename PrecT<P>::TA;
    constexpr int NF = Q * 3 * K;  // face values per lane and face (all components)
    // Face values at the Gauss points, entry (mu*3 + v)*K + comp, v = value,
    // d/dxi, d/deta.  The doubled edge fluxes of node mu, entry sk*K + comp
    // (sk = u, v, w flux), are written over the face values they come from:
    // x-edge l over sxR[mu*3*K + .][l], y-edge l over syB[mu*3*K + .][l].
    // Only the thread of that edge point reads those face values, and it
    // reads them all before it writes; the residual of component c reads
    // only entries of component c, which the next row's reconstruction
    // rewrites in the same wave, so no other wave can overwrite a flux
    // before it is read.
    __shared__ T sxR[NF][64], sxL[NF][64], syB[NF][64], syT[NF][64];
    auto FX = [&](int mu, int k, int l) -> T& { return sxR[mu * 3 * K + k][l]; };
    auto FY = [&](int mu, int k, int l) -> T& { return syB[mu * 3 * K + k][l]; };
    __shared__ double smx[K], smy[K];  // stage 3: per-wave maxima of the wave speeds
    __shared__ long long sbad[K];      // stage 3: per-wave first non-admissible cell

    const int lane = threadIdx.x & 63;
    // component of this wave (uniform: the plane pointers stay in SGPRs)
    const int c = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const Scheme& sch = a.sch;
    const int squared = sch.weights == W_BETA2 || (sch.weights == W_PAPER);
    const Flux<T, FLUX, K, 0> FXf(sch);
    const Flux<T, FLUX, K, 1> FYf(sch);
    const Tile2D* tiles = (const Tile2D*)a.tiles + a.tile_offset;

    // Stage 3 also gathers the wave speeds of the state it writes (for the
    // next step's flux and time step), after each tile's march: the gather
    // reads the tile's new averages back (they are in the L2 the stores
    // went through) with every wave, so the march itself carries no extra
    // registers and no wave waits for another's gather at a barrier.
    constexpr bool fuse_alpha = mode == MODE_S3;

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
        const int gi = tile.i0 - 2 + lane;          // this lane's column
        const int li = bc_map(gi, nx, bcx);         // column it reads
        const bool out_col = lane >= 2 && lane < 62 && gi < nx;

        // Every pointer of the march is formed here, once per tile: fields of
        // the problem table read inside the row loop would be reloaded after
        // each store (possible aliasing) and waited for with every load in
        // flight, the row-ahead prefetch included.
        const int64_t off_u = P_.off_u, off_d = P_.off_d;
        const TU* Uu = (const TU*)a.in.u + off_u + c * plane;
        const TD* Uv = (const TD*)a.in.d + off_d + c * plane;
        const TD* Uw = (const TD*)a.in.d + off_d + (K + c) * plane;
        const TU* Un = (const TU*)a.un + off_u + c * plane;     // stages 2, 3: U^n
        TD* Hv = (TD*)a.h + off_d + c * plane;                  // saved derivatives
        TD* Hw = (TD*)a.h + off_d + (K + c) * plane;
        TU* Ou = (TU*)a.out.u + off_u + c * plane;
        TD* Ov = (TD*)a.out.d + off_d + c * plane;
        TD* Ow = (TD*)a.out.d + off_d + (K + c) * plane;

        auto row_ptr = [&](int j) { return (uint32_t)(bc_map(j, ny, bcy) * nx + li); };
        // Solid walls: in a mirror image across x the x momentum (component
        // 1) is odd and the other averages even, and v-bar has the opposite
        // parity of its quantity; across y likewise with component 2 and
        // w-bar.  Signs of this lane's column, and of a row.
        const bool mx = FLUX == F_EULER && wall_mirrored(gi, nx, bcx);
        const bool nux = mx && c == 1, nvx = mx && c != 1, nwx = mx && c == 1;
        auto load_row = [&](int j, TU& u, TD& v, TD& w) {
            const uint32_t o = row_ptr(j);
            const bool my = FLUX == F_EULER && wall_mirrored(j, ny, bcy);
            const bool nuy = my && c == 2, nvy = my && c == 2, nwy = my && c != 2;
            u = neg_if(plane_at(Uu, o), nux != nuy);
            v = neg_if(plane_at(Uv, o), nvx != nvy);
            w = neg_if(plane_at(Uw, o), nwx != nwy);
        };
        const int j0 = tile.j0, jend = tile.j0 + tile.nrows;  // outputs j0..jend-1

        TU um, u0, up, un_;
        TD vm, v0, vp, vn_, wm, w0, wp, wn_;
        load_row(j0 - 2, um, vm, wm);
        load_row(j0 - 1, u0, v0, w0);
        load_row(j0, up, vp, wp);
        constexpr bool SYMD = sizeof(T) == 4 && (std::is_same<TU, double>::value || std::is_same<TU, float>::value);
        T dneg = 0;
        if constexpr (SYMD) dneg = (T)(u0 - um);
        T ytop[Q][3];            // top-face values of the previous row (this lane, comp)
        // previous row's flux sums: x differences and y sums of the
        // cell-average fluxes in the accumulation type, of the derivative
        // fluxes in T.  The FP64 path (PARTIAL) carries instead the part of
        // the previous row's residual known before its top edge (its x
        // difference less its bottom edge, in xdu_prev and xdd_prev): three
        // register pairs fewer through the march.  (In single precision
        // that form would round the sum of two large terms instead of their
        // small difference.)
        constexpr bool PARTIAL = P == P_F64;
        TA xdu_prev = 0, gyu_prev = 0;
        T xdd_prev[2] = {0, 0}, gyd_prev[2] = {0, 0};
        T hat_prev[2] = {0, 0};

        for (int r = j0 - 1; r <= jend; ++r) {
            // prefetch the row two above and the RK inputs of the output row
            load_row(r + 2, un_, vn_, wn_);
            TA unr = 0;
            T hvr = 0, hwr = 0;
            const bool emit = r > j0 && out_col;   // row r-1 is an output row
            const uint32_t oo = (uint32_t)((r - 1) * nx + gi);  // output row r-1 (in range if emit)
            if (mode == MODE_S2 || mode == MODE_S3) {
                // unconditional (lanes without output read element 0) so that
                // the loads stay in flight until the epilogue uses them
                const uint32_t ol = emit ? oo : 0u;
                unr = (TA)plane_at(Un, ol);
                hvr = (T)plane_at(Hv, ol);
                hwr = (T)plane_at(Hw, ol);
            }

            // ---- R: reconstruct cell (gi, r), component c -------------------
            if (r > j0 - 1) {
#pragma unroll
                for (int mu = 0; mu < Q; ++mu)
#pragma unroll
                    for (int v = 0; v < 3; ++v) syT[(mu * 3 + v) * K + c][lane] = ytop[mu][v];
            }
            T q[17];
            if constexpr (sizeof(T) == 4) {
                // Single precision: the column's own differences and the
                // differences of the side neighbours' averages from the centre
                // are rounded once from the wide averages; a corner is the sum
                // of the neighbour column's own difference and that column's
                // centre difference, which the compiler forms in one add with a
                // DPP lane shift on its first operand.
                const TU uc = u0;
                const T dp = (T)(up - uc), dr = (T)(from_right(u0) - uc);
                T dm, dl;
                if constexpr (SYMD) {
                    dm = -dneg;
                    dl = -from_left(dr);
                    dneg = dp;
                } else {
                    dm = (T)(um - uc);
                    dl = (T)(from_left(u0) - uc);
                }
                q[0] = from_left(dm) + dl;
                q[1] = dm;
                q[2] = from_right(dm) + dr;
                q[3] = dl;
                q[4] = (T)0;
                q[5] = dr;
                q[6] = from_left(dp) + dl;
                q[7] = dp;
                q[8] = from_right(dp) + dr;
            } else {
                const TU uc = u0;
                q[0] = (T)(from_left(um) - uc);
                q[1] = (T)(um - uc);
                q[2] = (T)(from_right(um) - uc);
                q[3] = (T)(from_left(u0) - uc);
                q[4] = (T)0;
                q[5] = (T)(from_right(u0) - uc);
                q[6] = (T)(from_left(up) - uc);
                q[7] = (T)(up - uc);
                q[8] = (T)(from_right(up) - uc);
            }
            {
                q[9] = (T)from_left(v0);
                q[10] = (T)from_right(v0);
                q[11] = (T)vm;
                q[12] = (T)vp;
                q[13] = (T)from_left(w0);
                q[14] = (T)from_right(w0);
                q[15] = (T)wm;
                q[16] = (T)wp;
            }
            T C[15], vhat, what;
            reconstruct2d<T>(q, sch, squared, C, vhat, what);
            const T ucT = (T)u0;
            {
                T val[2][Q], dn[2][Q], dtg[2][Q];
                // Derivatives go to the faces in local units (d/dxi, d/deta): the
                // edge flux is linear in them, so the 1/dx, 1/dy of u_x, u_y are
                // applied once to the residual instead of at every face point.
                face_values<T, Q>(C, val, dn, dtg);   // x-faces: dn = d/dxi, dt = d/deta
#pragma unroll
                for (int mu = 0; mu < Q; ++mu) {
                    sxL[(mu * 3 + 0) * K + c][lane] = ucT + val[0][mu];
                    sxL[(mu * 3 + 1) * K + c][lane] = dn[0][mu];
                    sxL[(mu * 3 + 2) * K + c][lane] = dtg[0][mu];
                    sxR[(mu * 3 + 0) * K + c][lane] = ucT + val[1][mu];
                    sxR[(mu * 3 + 1) * K + c][lane] = dn[1][mu];
                    sxR[(mu * 3 + 2) * K + c][lane] = dtg[1][mu];
                }
                T D[15];
                transpose15(C, D);
                face_values<T, Q>(D, val, dn, dtg);   // y-faces: dn = d/deta, dt = d/dxi
#pragma unroll
                for (int mu = 0; mu < Q; ++mu) {
                    syB[(mu * 3 + 0) * K + c][lane] = ucT + val[0][mu];
                    syB[(mu * 3 + 1) * K + c][lane] = dtg[0][mu];
                    syB[(mu * 3 + 2) * K + c][lane] = dn[0][mu];
                    ytop[mu][0] = ucT + val[1][mu];
                    ytop[mu][1] = dtg[1][mu];
                    ytop[mu][2] = dn[1][mu];
                }
            }

            if (r > j0 - 1) {
                __syncthreads();  // A: face values of row r (and top faces of r-1) ready
                // ---- F: edge fluxes ---------------------------------------
                for (int sl = threadIdx.x; sl < 2 * Q * 64; sl += 64 * K) {
                    const int kind = sl / (Q * 64);
                    const int mu = (sl >> 6) % Q;
                    const int l = sl & 63;
                    if constexpr (P == P_F64 && FLUX == F_EULER && K == 4) {
                        // one side at a time, and within a side the flux and
                        // its two Jacobian-vector products one after the
                        // other, each from its own four face values: fewer
                        // registers at the register peak of the FP64 march
                        T out[3 * K];
                        auto side = [&](auto& F, T (*src)[64], int ll, T al, bool first) {
                            const int b = mu * 3 * K;
                            T U[K], D[K], o[K];
#pragma unroll
                            for (int k = 0; k < K; ++k) U[k] = src[b + k][ll];
                            const auto w = F.prim(U);
                            F.flux(U, w, o);
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                const T ok = o[k] + al * U[k];
                                out[k] = first ? ok : out[k] + ok;
                            }
#pragma unroll
                            for (int sk = 1; sk < 3; ++sk) {
#pragma unroll
                                for (int k = 0; k < K; ++k) D[k] = src[b + sk * K + k][ll];
                                F.jvp(w.u, w.v, w.q2h, w.H, D, o);
#pragma unroll
                                for (int k = 0; k < K; ++k) {
                                    const T ok = o[k] + al * D[k];
                                    out[sk * K + k] = first ? ok : out[sk * K + k] + ok;
                                }
                            }
                        };
                        if (kind == 0) {
                            if (l < 63) {   // x-edge between lanes l and l+1
                                side(FXf, sxR, l, ax, true);
                                side(FXf, sxL, l + 1, -ax, false);
#pragma unroll
                                for (int k = 0; k < 3 * K; ++k) FX(mu, k, l) = out[k];
                            }
                        } else {            // y-edge between rows r-1 and r, column l
                            side(FYf, syT, l, ay, true);
                            side(FYf, syB, l, -ay, false);
#pragma unroll
                            for (int k = 0; k < 3 * K; ++k) FY(mu, k, l) = out[k];
                        }
                        continue;
                    }
                    T UL[K], VL[K], WL[K], UR[K], VR[K], WR[K], out[3 * K];
                    if (kind == 0) {
                        if (l < 63) {   // x-edge between lanes l and l+1
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                UL[k] = sxR[(mu * 3 + 0) * K + k][l];
                                VL[k] = sxR[(mu * 3 + 1) * K + k][l];
                                WL[k] = sxR[(mu * 3 + 2) * K + k][l];
                                UR[k] = sxL[(mu * 3 + 0) * K + k][l + 1];
                                VR[k] = sxL[(mu * 3 + 1) * K + k][l + 1];
                                WR[k] = sxL[(mu * 3 + 2) * K + k][l + 1];
                            }
                            lf_edge<T, FLUX, K, 0>(FXf, UL, VL, WL, UR, VR, WR, ax, out);
#pragma unroll
                            for (int k = 0; k < 3 * K; ++k) FX(mu, k, l) = out[k];
                        }
                    } else {            // y-edge between rows r-1 and r, column l
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            UL[k] = syT[(mu * 3 + 0) * K + k][l];
                            VL[k] = syT[(mu * 3 + 1) * K + k][l];
                            WL[k] = syT[(mu * 3 + 2) * K + k][l];
                            UR[k] = syB[(mu * 3 + 0) * K + k][l];
                            VR[k] = syB[(mu * 3 + 1) * K + k][l];
                            WR[k] = syB[(mu * 3 + 2) * K + k][l];
                        }
                        lf_edge<T, FLUX, K, 1>(FYf, UL, VL, WL, UR, VR, WR, ay, out);
#pragma unroll
                        for (int k = 0; k < 3 * K; ++k) FY(mu, k, l) = out[k];
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
                        fr += w * FX(mu, sk * K + c, lane);
                        if constexpr (P != P_F64)
                            fl += w * FX(mu, sk * K + c, lane > 0 ? lane - 1 : 0);
                        g += w * FY(mu, sk * K + c, lane);
                    }
                    // FP64: the left edge's sum is the left lane's right-edge
                    // sum, the same bits, taken by a lane shift instead of
                    // further LDS reads (the FP64 march is LDS-heavy)
                    if constexpr (P == P_F64) fl = from_left(fr);
                    if (sk == 0) {
                        xdu = (TA)fr - (TA)fl;
                        gyu = (TA)g;
                    } else {
                        xdd[sk - 1] = fr - fl;
                        gyd[sk - 1] = g;
                    }
                }
                if (r > j0) {
                    // v- and w-fluxes carry the derivatives in local units
                    TA Lu;
                    T Lv, Lw;
                    if constexpr (PARTIAL) {
                        Lu = -(xdu_prev + gyu * inv_dy_a);
                        Lv = -inv_dx * (xdd_prev[0] + rx * gyd[0]);
                        Lw = -inv_dy * (xdd_prev[1] + gyd[1]);
                    } else {
                        Lu = -(xdu_prev * inv_dx_a + (gyu - gyu_prev) * inv_dy_a);
                        Lv = -inv_dx * (xdd_prev[0] + rx * (gyd[0] - gyd_prev[0]));
                        Lw = -inv_dy * (ry * xdd_prev[1] + (gyd[1] - gyd_prev[1]));
                    }
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
                                plane_at(Ou, oo) = (TU)(ucur + dta * Lu);
                                plane_at(Ov, oo) = (TD)(hat_prev[0] + dtt * Lv);
                                plane_at(Ow, oo) = (TD)(hat_prev[1] + dtt * Lw);
                                plane_at(Hv, oo) = (TD)hat_prev[0];
                                plane_at(Hw, oo) = (TD)hat_prev[1];
                            } else if (mode == MODE_S2) {
                                plane_at(Ou, oo) = (TU)((TA)0.75 * unr + (TA)0.25 * (ucur + dta * Lu));
                                plane_at(Ov, oo) = (TD)((T)0.75 * hvr + (T)0.25 * (hat_prev[0] + dtt * Lv));
                                plane_at(Ow, oo) = (TD)((T)0.75 * hwr + (T)0.25 * (hat_prev[1] + dtt * Lw));
                            } else {
                                const TA third = (TA)(1.0 / 3.0), two3 = (TA)(2.0 / 3.0);
                                plane_at(Ou, oo) = (TU)(third * unr + two3 * (ucur + dta * Lu));
                                plane_at(Ov, oo) = (TD)((T)(1.0 / 3.0) * hvr +
                                              (T)(2.0 / 3.0) * (hat_prev[0] + dtt * Lv));
                                plane_at(Ow, oo) = (TD)((T)(1.0 / 3.0) * hwr +
                                              (T)(2.0 / 3.0) * (hat_prev[1] + dtt * Lw));
                            }
                        }
                    }
                }
                if constexpr (PARTIAL) {
                    xdu_prev = xdu * inv_dx_a - gyu * inv_dy_a;
                    xdd_prev[0] = xdd[0] - rx * gyd[0];
                    xdd_prev[1] = ry * xdd[1] - gyd[1];
                } else {
                    xdu_prev = xdu;
                    gyu_prev = gyu;
#pragma unroll
                    for (int sk = 0; sk < 2; ++sk) {
                        xdd_prev[sk] = xdd[sk];
                        gyd_prev[sk] = gyd[sk];
                    }
                }
            }
            hat_prev[0] = vhat;
            hat_prev[1] = what;
            // advance the register window one row up
            um = u0; u0 = up; up = un_;
            vm = v0; v0 = vp; vp = vn_;
            wm = w0; w0 = wp; wp = wn_;
        }
        __syncthreads();  // LDS reuse by the next tile; the tile's stores are visible
        if (fuse_alpha)
            gather_tile_speeds<TU, FLUX, K>((const TU*)a.out.u + off_u, (uint32_t)plane, nx, tile.i0,
                                            j0, jend, a.probs[tile.prob], sch, smx, smy, sbad);
    }
}

// Launches the stage kernel of one precision: Euler in either register
// variant, the scalar laws in variant 0.
template <int P, int K, int Q, int FLUX, int V>
void stage2d_launch_modes(int mode, const StageArgs& a, int grid, hipStream_t s) {
    constexpr int threads = 64 * K;
    switch (mode) {
        case MODE_RHS: stage2d_kernel<P, K, Q, FLUX, MODE_RHS, V><<<grid, threads, 0, s>>>(a); break;
        case MODE_S1: stage2d_kernel<P, K, Q, FLUX, MODE_S1, V><<<grid, threads, 0, s>>>(a); break;
        case MODE_S2: stage2d_kernel<P, K, Q, FLUX, MODE_S2, V><<<grid, threads, 0, s>>>(a); break;
        default: stage2d_kernel<P, K, Q, FLUX, MODE_S3, V><<<grid, threads, 0, s>>>(a); break;
    }
}

template <int P>
hipError_t stage2d_launch_prec(int flux, int Q, int mode, int variant, const StageArgs& a,
                               int grid, hipStream_t s) {
    if (flux == F_EULER) {
        if (Q == 2) {
            if (variant) stage2d_launch_modes<P, 4, 2, F_EULER, 1>(mode, a, grid, s);
            else stage2d_launch_modes<P, 4, 2, F_EULER, 0>(mode, a, grid, s);
        } else {
            if (variant) stage2d_launch_modes<P, 4, 3, F_EULER, 1>(mode, a, grid, s);
            else stage2d_launch_modes<P, 4, 3, F_EULER, 0>(mode, a, grid, s);
        }
    } else if (flux == F_BURGERS) {
        if (Q == 2) stage2d_launch_modes<P, 1, 2, F_BURGERS, 0>(mode, a, grid, s);
        else stage2d_launch_modes<P, 1, 3, F_BURGERS, 0>(mode, a, grid, s);
    } else {
        if (Q == 2) stage2d_launch_modes<P, 1, 2, F_ADV, 0>(mode, a, grid, s);
        else stage2d_launch_modes<P, 1, 3, F_ADV, 0>(mode, a, grid, s);
    }
    return hipGetLastError();
}

}  // namespace hweno

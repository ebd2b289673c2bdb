// Device-side building blocks of the HWENO stage kernels (gfx950, wave64):
// precision policies, boundary index maps, physical fluxes and their
// Jacobian-vector products, and the nonlinear weights.
#pragma once

#include "ff.h"
#include "internal.h"

namespace hweno {

// ---------------------------------------------------------------- types ----

// TU: storage of cell averages; TD: storage of derivative averages;
// T: reconstruction / flux arithmetic; TA: arithmetic of the cell-average
// update (flux differences and the RK combination of u-bar).
template <int P> struct PrecT;
template <> struct PrecT<P_F64> { using TU = double; using TD = double; using T = double; using TA = double; };
template <> struct PrecT<P_F32> { using TU = float;  using TD = float;  using T = float;  using TA = float; };
template <> struct PrecT<P_ACC64> { using TU = double; using TD = float; using T = float; using TA = double; };
template <> struct PrecT<P_KAHAN> { using TU = ffs; using TD = float; using T = float; using TA = ff; };

// Ghost cells as index maps: periodic wraps, transmissive clamps to the
// nearest interior cell (every unknown of a ghost cell is that cell's),
// reflective mirrors (with the signs of wall_mirrored below).
// Interior indices map to themselves under every condition; they are tested
// first because the integer remainder has no scalar instruction and costs
// about thirty vector instructions even for a wave-uniform row index.
__device__ __forceinline__ int bc_map(int i, int n, int bc) {
    if (i >= 0 && i < n) return i;
    if (bc == BC_PERIODIC) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    if (bc == BC_REFLECTIVE) {   // mirror images across both walls (period 2n)
        int r = i % (2 * n);
        if (r < 0) r += 2 * n;
        return r < n ? r : 2 * n - 1 - r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// True where index i lies in a mirror image of the domain across a solid
// wall (an odd number of reflections): there the normal momentum is odd and
// every other conserved quantity even, and the derivative mean along the
// wall normal has the opposite parity of its quantity.
__device__ __forceinline__ bool wall_mirrored(int i, int n, int bc) {
    if (bc != BC_REFLECTIVE || (i >= 0 && i < n)) return false;
    int r = i % (2 * n);
    if (r < 0) r += 2 * n;
    return r >= n;
}

template <class V> __device__ __forceinline__ V neg_if(V x, bool neg) { return neg ? -x : x; }

__device__ __forceinline__ double as_double(uint64_t b) { return __longlong_as_double((long long)b); }

// Element idx of one plane of a problem (at most 2^29 cells of at most 8
// bytes, so byte offsets fit in 32 bits): a wave-uniform base plus a 32-bit
// offset, which the global memory instructions take as an SGPR base and a
// VGPR offset, so that no lane forms a 64-bit address.
template <class X> __device__ __forceinline__ X& plane_at(X* base, uint32_t idx) {
    return *reinterpret_cast<X*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(X));
}
template <class X> __device__ __forceinline__ const X& plane_at(const X* base, uint32_t idx) {
    return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) +
                                       idx * (uint32_t)sizeof(X));
}

// Whole-wave lane shifts through DPP (wave_shr:1 / wave_shl:1 of the GFX9
// data-parallel primitives): lane l receives lane l-1 (from_left) or lane l+1
// (from_right); the lane at the end of the wave, which has no source, gets 0
// (bound_ctrl), so the shift is a single v_mov_b32_dpp.  Callers never use the
// end lanes' results.
template <int CTRL> __device__ __forceinline__ int dpp_shift(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;
template <int CTRL> __device__ __forceinline__ float dpp_shift(float v) {
    return __int_as_float(dpp_shift<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double dpp_shift(double v) {
    const int lo = dpp_shift<CTRL>(__double2loint(v));
    const int hi = dpp_shift<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int CTRL> __device__ __forceinline__ ffs dpp_shift(ffs v) {
    ffs r;
    r.hi = dpp_shift<CTRL>(v.hi);
    r.lo = dpp_shift<CTRL>(v.lo);
    return r;
}
template <class T> __device__ __forceinline__ T from_left(T v) { return dpp_shift<DPP_WAVE_SHR1>(v); }
template <class T> __device__ __forceinline__ T from_right(T v) { return dpp_shift<DPP_WAVE_SHL1>(v); }

// Reciprocals: v_rcp_f32 (1 ulp) in single precision; in double precision
// v_rcp_f64 refined by two Newton steps, r <- r + r (1 - x r), to within an
// ulp or two of the correctly rounded quotient.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// ------------------------------------------------------- physical fluxes ---
//
// For a state U and a derivative direction V of one side of an interface,
// side() returns F(U) and the Jacobian-vector products (dF/dU) V and
// (dF/dU) W: the fluxes of the differentiated system h = f'(u) v (Sec. 2.1)
// and f^v, f^w / g^v, g^w (eq. 2D-uvw-cartesian).  DIR 0 = x, 1 = y.

template <class T, int FLUX, int K, int DIR> struct Flux;

template <class T, int DIR> struct Flux<T, F_ADV, 1, DIR> {
    T a;
    __device__ Flux(const Scheme& s) : a((T)s.adv[DIR]) {}
    __device__ __forceinline__ void side(const T* U, const T* V, const T* W, T* f, T* fv,
                                         T* fw) const {
        f[0] = a * U[0];
        fv[0] = a * V[0];
        if (W) fw[0] = a * W[0];
    }
};

template <class T, int DIR> struct Flux<T, F_BURGERS, 1, DIR> {
    __device__ Flux(const Scheme&) {}
    __device__ __forceinline__ void side(const T* U, const T* V, const T* W, T* f, T* fv,
                                         T* fw) const {
        f[0] = (T)0.5 * U[0] * U[0];
        fv[0] = U[0] * V[0];
        if (W) fw[0] = U[0] * W[0];
    }
};

// 1D Euler, U = (rho, rho*mu, E).
template <class T> struct Flux<T, F_EULER, 3, 0> {
    T gm1;
    __device__ Flux(const Scheme& s) : gm1((T)(s.gas_gamma - 1.0)) {}
    __device__ __forceinline__ void side(const T* U, const T* V, const T*, T* f, T* fv,
                                         T*) const {
        const T rho = U[0], m = U[1], E = U[2];
        const T ir = rcp(rho);
        const T u = m * ir;
        const T half_u2 = (T)0.5 * u * u;
        const T p = gm1 * (E - rho * half_u2);
        const T Ep = E + p;
        const T H = Ep * ir;
        f[0] = m;
        f[1] = m * u + p;
        f[2] = u * Ep;
        const T dr = V[0], dm = V[1], dE = V[2];
        const T dp = gm1 * (dE - u * dm + half_u2 * dr);
        // the rows of A V with the common factor a = dm - u dr taken out:
        // 2u dm - u^2 dr = u (dm + a), H dm - u H dr = H a
        const T a = dm - u * dr;
        fv[0] = dm;
        fv[1] = u * (dm + a) + dp;
        fv[2] = H * a + u * (dE + dp);
    }
};

// 2D Euler, U = (rho, rho*mu, rho*nu, E); DIR selects F (x) or G (y).
template <class T, int DIR> struct Flux<T, F_EULER, 4, DIR> {
    T gm1;
    __device__ Flux(const Scheme& s) : gm1((T)(s.gas_gamma - 1.0)) {}
    // (dF/dU) D or (dG/dU) D, with the common factor of three of its rows
    // taken out: for F, a = dm - u dr gives 2u dm - u^2 dr = u (dm + a),
    // v dm + u dn - uv dr = v a + u dn and H dm - uH dr = H a (for G
    // likewise with b = dn - v dr)
    __device__ __forceinline__ void jvp(T u, T v, T q2h, T H, const T* D, T* out) const {
        const T dr = D[0], dm = D[1], dn = D[2], dE = D[3];
        const T dp = gm1 * (dE - u * dm - v * dn + q2h * dr);
        if (DIR == 0) {
            const T a = dm - u * dr;
            out[0] = dm;
            out[1] = u * (dm + a) + dp;
            out[2] = v * a + u * dn;
            out[3] = H * a + u * (dE + dp);
        } else {
            const T b = dn - v * dr;
            out[0] = dn;
            out[1] = u * b + v * dm;
            out[2] = v * (dn + b) + dp;
            out[3] = H * b + v * (dE + dp);
        }
    }
    // velocity, half its square, pressure and total enthalpy of U
    struct Prim {
        T u, v, q2h, p, H;
    };
    __device__ __forceinline__ Prim prim(const T* U) const {
        const T rho = U[0], m = U[1], n = U[2], E = U[3];
        const T ir = rcp(rho);
        const T u = m * ir, v = n * ir;
        const T q2h = (T)0.5 * (u * u + v * v);
        const T p = gm1 * (E - rho * q2h);
        return {u, v, q2h, p, (E + p) * ir};
    }
    __device__ __forceinline__ void flux(const T* U, const Prim& w, T* f) const {
        const T m = U[1], n = U[2], Ep = U[3] + w.p;
        if (DIR == 0) {
            f[0] = m; f[1] = m * w.u + w.p; f[2] = m * w.v; f[3] = w.u * Ep;
        } else {
            f[0] = n; f[1] = n * w.u; f[2] = n * w.v + w.p; f[3] = w.v * Ep;
        }
    }
    __device__ __forceinline__ void side(const T* U, const T* V, const T* W, T* f, T* fv,
                                         T* fw) const {
        const Prim w = prim(U);
        flux(U, w, f);
        jvp(w.u, w.v, w.q2h, w.H, V, fv);
        jvp(w.u, w.v, w.q2h, w.H, W, fw);
    }
};

// ------------------------------------------------------------ wave speeds --
//
// |f'(u)| and |g'(u)| at the cell average U (Euler: |velocity| + sound
// speed), in double precision with no contraction and IEEE divisions, so
// that every kernel that evaluates it produces the same bits, and the same
// bits as a plain evaluation of the definition (time steps then agree
// exactly with a reference run, also along trajectories that end in a
// non-admissible state); returns false if U is not finite or (Euler)
// rho <= 0 or p <= 0 (sx, sy are then meaningless).  Straight-line code: the
// sound speed is evaluated whatever the admissibility test says and selected
// afterwards, so that a caller can schedule the chain with other work.
template <int FLUX, int DIM, int K>
__device__ __forceinline__ bool wave_speed(const double* u, const Scheme& sch, double& sx,
                                           double& sy) {
#pragma clang fp contract(off)
    bool ok = true;
#pragma unroll
    for (int c = 0; c < K; ++c) ok = ok & (bool)isfinite(u[c]);
    if (FLUX == F_ADV) {
        sx = fabs(sch.adv[0]);
        sy = fabs(sch.adv[1]);
    } else if (FLUX == F_BURGERS) {
        sx = sy = fabs(u[0]);
    } else {
        const double g = sch.gas_gamma;
        const double rho = u[0];
        const double vx = u[1] / rho;
        const double vy = DIM == 2 ? u[2] / rho : 0.0;
        const double ke = 0.5 * rho * (vx * vx + vy * vy);
        const double pr = (g - 1.0) * (u[K - 1] - ke);
        ok = ok & (rho > 0.0) & (pr > 0.0);
        const double cs2 = g * pr / rho;
        const double cs = sqrt(ok ? cs2 : 1.0);
        sx = fabs(vx) + cs;
        sy = fabs(vy) + cs;
    }
    return ok;
}

// Maximum over the wave of a non-negative double, returned to every lane:
// DPP steps within quads, half rows and rows, then the row broadcasts of the
// GFX9 data-parallel primitives (row_bcast:15 into rows 1 and 3, then
// row_bcast:31 into rows 2 and 3) leave it in lane 63, which is read out.
// Lanes a broadcast does not write see 0, which leaves a non-negative
// maximum as it is.  (An xor butterfly through ds_bpermute costs LDS round
// trips and more instructions.)
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_or_zero(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xF, ROWS == 0xF),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xF, ROWS == 0xF));
}
__device__ __forceinline__ double max_of(double a, double b) { return b > a ? b : a; }
__device__ __forceinline__ double wave_max_d(double v) {
    v = max_of(v, dpp_or_zero<0xB1, 0xF>(v));    // quad_perm [1,0,3,2]
    v = max_of(v, dpp_or_zero<0x4E, 0xF>(v));    // quad_perm [2,3,0,1]
    v = max_of(v, dpp_or_zero<0x141, 0xF>(v));   // row_half_mirror
    v = max_of(v, dpp_or_zero<0x140, 0xF>(v));   // row_mirror
    v = max_of(v, dpp_or_zero<0x142, 0xA>(v));   // row_bcast:15
    v = max_of(v, dpp_or_zero<0x143, 0xC>(v));   // row_bcast:31
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

__device__ __forceinline__ long long wave_min_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const long long w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// Speeds only grow during a launch and their slots start at zero, so any
// relaxed read of a slot during the launch is a lower bound of its final
// value: a block maximum that does not exceed it has nothing to add, and most
// blocks skip the atomic (every block of a problem targets the same address,
// where atomics serialize).  Callers read the slot (peek_slot) some time
// before they publish, so that the read's latency overlaps their work.
__device__ __forceinline__ uint64_t peek_slot(const uint64_t* slot) {
    return __hip_atomic_load(const_cast<uint64_t*>(slot), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void publish_max(uint64_t* slot, double v, uint64_t seen) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b > seen) atomicMax((unsigned long long*)slot, b);
}

// Folds reduced speeds and a first bad cell into the problem's slots for the
// state being written (one lane calls this; seen_x, seen_y: earlier reads of
// the two slots).  Speeds are non-negative, so their bit patterns order as
// unsigned integers.
__device__ __forceinline__ void publish_reduced(ProbDev& P, double mx, double my, long long bad,
                                                uint64_t seen_x, uint64_t seen_y) {
    publish_max(&P.ax_next, mx, seen_x);
    if (my > 0.0) publish_max(&P.ay_next, my, seen_y);
    if (bad != LLONG_MAX) {
        atomicMin((long long*)&P.bad_cell, bad);
        atomicOr(&P.err, ERR_STATE_BAD);
    }
}

// Wave-level version: every lane brings its values, lane 0 publishes.  The
// bad-cell minimum is only formed when some lane has one.
__device__ __forceinline__ void publish_next_speeds(ProbDev& P, double mx, double my,
                                                    long long bad, uint64_t seen_x,
                                                    uint64_t seen_y) {
    mx = wave_max_d(mx);
    my = wave_max_d(my);
    if (__any(bad != LLONG_MAX)) bad = wave_min_ll(bad);
    if ((threadIdx.x & 63) == 0) publish_reduced(P, mx, my, bad, seen_x, seen_y);
}

// Folds lane maxima of the wave speeds, and first non-admissible cells, of a
// workgroup into the problem's slots: reduced over each wave, then over the
// waves through LDS (s_mx, s_my, s_bad: one entry per wave) by thread 0,
// which read the slots (seen_x, seen_y) before the values were formed.
// Every thread of the workgroup calls it (it holds a barrier).
__device__ __forceinline__ void publish_tile_speeds(ProbDev& P, double mx, double my,
                                                    long long bad, uint64_t seen_x,
                                                    uint64_t seen_y, double* s_mx, double* s_my,
                                                    long long* s_bad) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    mx = wave_max_d(mx);
    my = wave_max_d(my);
    if (__any(bad != LLONG_MAX)) bad = wave_min_ll(bad);
    if (lane == 0) {
        s_mx[w] = mx;
        s_my[w] = my;
        s_bad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < nw; ++v) {
            mx = fmax(mx, s_mx[v]);
            my = fmax(my, s_my[v]);
            bad = s_bad[v] < bad ? s_bad[v] : bad;
        }
        publish_reduced(P, mx, my, bad, seen_x, seen_y);
    }
}

// Wave speeds of the cell averages a stage-3 launch has just written for one
// 2D tile (rows [j0, jend), output columns [i0, i0 + STRIP_OUT) within the
// problem), gathered after the tile's march by every wave of the workgroup:
// wave w reads a contiguous share of the rows (they come from the L2 the
// march's stores went through, or from HBM), lane l column i0 + l, and
// evaluates wave_speed exactly for each cell; the workgroup's maxima and
// first non-admissible cell are folded into the problem's slots for the next
// step.  out_u: the problem's u-bar planes of the state written; the march's
// stores must be visible (a barrier after them); s_mx, s_my, s_bad: LDS of
// one entry per wave.  Not inlined: its FP64 division chains would otherwise
// raise the register allocation of the whole march (and it stays within the
// registers a call may use without saving any: no scratch).
template <class TU, int FLUX, int K>
__device__ __attribute__((noinline)) void gather_tile_speeds(const TU* out_u, uint32_t plane, int nx,
                                                   int i0, int j0, int jend, ProbDev& P,
                                                   const Scheme& sch, double* s_mx, double* s_my,
                                                   long long* s_bad) {
    // the planes are global memory (global rather than flat loads) at
    // wave-uniform bases (scalar registers, 32-bit offsets per lane)
    using GC = const __attribute__((address_space(1))) char;
    auto uniform = [](uint64_t v) {
        return (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v) |
               ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32);
    };
    GC* gp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) gp[k] = (GC*)uniform((uint64_t)out_u + (uint64_t)k * plane * sizeof(TU));
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint64_t seen_x = 0, seen_y = 0;
    if (threadIdx.x == 0) {   // read early: the gather covers the latency
        seen_x = peek_slot(&P.ax_next);
        seen_y = peek_slot(&P.ay_next);
    }
    const bool col = lane < STRIP_OUT && i0 + lane < nx;
    const int per = (jend - j0 + nw - 1) / nw;
    const int ra = j0 + w * per, rb = min(jend, ra + per);
    const uint32_t ci = (uint32_t)(i0 + (col ? lane : 0));
    double mx = 0.0, my = 0.0;
    long long bad = LLONG_MAX;
    for (int j = ra; j < rb; ++j) {
        const uint32_t off = ((uint32_t)(j * nx) + ci) * (uint32_t)sizeof(TU);
        double u[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            TU v;
            if constexpr (sizeof(TU) == 8)
                v = __builtin_bit_cast(TU, *(const __attribute__((address_space(1))) uint64_t*)(gp[k] + off));
            else
                v = __builtin_bit_cast(TU, *(const __attribute__((address_space(1))) uint32_t*)(gp[k] + off));
            u[k] = (double)v;
        }
        if (col) {
            double sx, sy;
            if (wave_speed<FLUX, 2, K>(u, sch, sx, sy)) {
                mx = fmax(mx, sx);
                my = fmax(my, sy);
            } else {
                const long long b = (long long)j * nx + i0 + lane;
                bad = b < bad ? b : bad;
            }
        }
    }
    publish_tile_speeds(P, mx, my, bad, seen_x, seen_y, s_mx, s_my, s_bad);
}

// --------------------------------------- classical smoothness indicator ---
//
// The indicator the paper prints for comparison with its own (eq.
// smoothness-indicator-typical and its 2D form): in cell units, the sum over
// derivative orders >= 1 of the integrals over the cell of the squared
// derivatives.  For p = sum_i c_i xi^a_i eta^b_i it is the quadratic form
// sum_ij c_i c_j M_ij, M_ij = sum_(m,n) (a_i)_m (a_j)_m (b_i)_n (b_j)_n
// mu(a_i + a_j - 2m) mu(b_i + b_j - 2n), with (a)_m the falling factorial
// and mu(k) the k-th moment of [-1/2, 1/2].  The entries are evaluated at
// compile time.
namespace classical {
constexpr double moment(int k) {
    if (k % 2) return 0.0;
    double p = 1.0;
    for (int i = 0; i < k; ++i) p *= 0.5;
    return p / (k + 1);
}
constexpr double falling(int a, int m) {
    double r = 1.0;
    for (int i = 0; i < m; ++i) r *= (double)(a - i);
    return r;
}
constexpr double entry(int ai, int bi, int aj, int bj) {
    double s = 0.0;
    for (int m = 0; m <= 4; ++m)
        for (int n = 0; m + n <= 4; ++n) {
            if (m + n == 0 || m > ai || m > aj || n > bi || n > bj) continue;
            s += falling(ai, m) * falling(aj, m) * falling(bi, n) * falling(bj, n) *
                 moment(ai + aj - 2 * m) * moment(bi + bj - 2 * n);
        }
    return s;
}
// exponents of the 2D basis 1, xi, eta, xi^2, xi eta, eta^2, ... eta^4
constexpr int EX[15] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
constexpr int EY[15] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4};
template <int I, int J> struct E1 { static constexpr double v = entry(I, 0, J, 0); };
template <int I, int J> struct E2 {
    static constexpr double v = entry(EX[I], EY[I], EX[J], EY[J]);
};

template <class T, int I, int J>
__device__ __forceinline__ void acc1(const T* c, T& b) {
    if constexpr (I <= 4) {
        if constexpr (J <= 4) {
            constexpr double m = (I == J ? 1.0 : 2.0) * E1<I, J>::v;
            if constexpr (m != 0.0) b += (T)m * c[I] * c[J];
            acc1<T, I, J + 1>(c, b);
        } else {
            acc1<T, I + 1, I + 1>(c, b);
        }
    }
}
template <class T, int I, int J>
__device__ __forceinline__ void acc2(const T* c, T& b) {
    if constexpr (I <= 14) {
        if constexpr (J <= 14) {
            constexpr double m = (I == J ? 1.0 : 2.0) * E2<I, J>::v;
            if constexpr (m != 0.0) b += (T)m * c[I] * c[J];
            acc2<T, I, J + 1>(c, b);
        } else {
            acc2<T, I + 1, I + 1>(c, b);
        }
    }
}
}  // namespace classical

// indicator of a 1D quartic c[0..4] / 2D quartic c[0..14] (constant ignored)
template <class T> __device__ __forceinline__ T beta_classical_1d(const T* c) {
    T b = 0;
    classical::acc1<T, 1, 1>(c, b);
    return b;
}
template <class T> __device__ __forceinline__ T beta_classical_2d(const T* c) {
    T b = 0;
    classical::acc2<T, 1, 1>(c, b);
    return b;
}

// ------------------------------------------- characteristic variables ---
//
// Eigenvectors of the Euler flux Jacobian at a cell's own average, for the
// reconstruction in local characteristic variables (remark closing Sec.
// 2.2).  U = (rho, m_n, [m_t,] E) with m_n the momentum along the direction
// and m_t across it; columns of R (rows of L = R^-1) belong to the
// eigenvalues v_n - c, v_n, [v_n (shear),] v_n + c.
template <class T, int K> struct Eigen {
    // the entries are closed forms in these scalars; no matrix is stored, so
    // that rows picked by a run-time index stay in registers
    T vn, vt, c, H, hq2, b1, b2, ec, hb1;
    __device__ __forceinline__ Eigen(const T* U, T gm1) {
        const T ir = rcp(U[0]);
        vn = U[1] * ir;
        vt = K == 4 ? U[2] * ir : (T)0;
        hq2 = (T)0.5 * (vn * vn + vt * vt);
        const T p = gm1 * (U[K - 1] - U[0] * hq2);
        const T c2 = (gm1 + (T)1) * p * ir;
        c = sqrt(c2);
        const T ic = rcp(c);
        H = (U[K - 1] + p) * ir;
        b1 = gm1 * ic * ic;
        b2 = b1 * hq2;
        ec = (T)0.5 * ic;
        hb1 = (T)0.5 * b1;
    }
    // L[i][k] (row i: field, column k: component), constant indices
    __device__ __forceinline__ T L(int i, int k) const {
        if (K == 3) {
            if (i == 1) return k == 0 ? (T)1 - b2 : (k == 1 ? b1 * vn : -b1);
            const T s = i == 0 ? (T)1 : (T)-1;   // fields v-c (0) and v+c (2)
            return k == 0 ? (T)0.5 * b2 + s * vn * ec : (k == 1 ? -(hb1 * vn) - s * ec : hb1);
        }
        if (i == 1) return k == 0 ? (T)1 - b2 : (k == 1 ? b1 * vn : (k == 2 ? b1 * vt : -b1));
        if (i == 2) return k == 0 ? -vt : (k == 2 ? (T)1 : (T)0);
        const T s = i == 0 ? (T)1 : (T)-1;       // fields v-c (0) and v+c (3)
        return k == 0 ? (T)0.5 * b2 + s * vn * ec
                      : (k == 1 ? -(hb1 * vn) - s * ec : (k == 2 ? -hb1 * vt : hb1));
    }
    // R[i][k] (row i: component, column k: field), constant indices
    __device__ __forceinline__ T R(int i, int k) const {
        const int kc = K == 3 ? (k == 2 ? 3 : k) : k;   // 1D has no shear field
        if (i == 0) return kc == 2 ? (T)0 : (T)1;
        if (i == 1) return kc == 0 ? vn - c : (kc == 3 ? vn + c : (kc == 1 ? vn : (T)0));
        if (K == 4 && i == 2) return kc == 2 ? (T)1 : vt;
        return kc == 0 ? H - vn * c : (kc == 3 ? H + vn * c : (kc == 1 ? hq2 : vt));
    }
    // row i of L or of R for a run-time (wave-uniform) i
    __device__ __forceinline__ void lrow(int i, T* out) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            T v = L(K - 1, k);
#pragma unroll
            for (int j = K - 2; j >= 0; --j) v = i == j ? L(j, k) : v;
            out[k] = v;
        }
    }
    __device__ __forceinline__ void rrow(int i, T* out) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            T v = R(K - 1, k);
#pragma unroll
            for (int j = K - 2; j >= 0; --j) v = i == j ? R(j, k) : v;
            out[k] = v;
        }
    }
    // w = L x and x = R w (vectors in the (rho, m_n, [m_t,] E) order)
    __device__ __forceinline__ void left(const T* x, T* w) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            T a = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) a += L(k, j) * x[j];
            w[k] = a;
        }
    }
    __device__ __forceinline__ void right(const T* w, T* x) const {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            T a = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) a += R(i, k) * w[k];
            x[i] = a;
        }
    }
};

// ----------------------------------------------------- nonlinear weights ---
//
// omega~_m = gamma_m (1 + tau^2 / D_m), omega = omega~ / sum (eq.
// nonlinear-weights, eq. nonlinear-weights-2D), with D_m = beta_m + eps or
// beta_m^2 + eps (SQ = 1) or chosen per value (SQ = -1, from `squared`),
// tau = mean_m |beta_0 - beta_m|.
template <class T, int M, int SQ>
__device__ __forceinline__ void nonlinear_weights_form(const T* beta, const Scheme& s, int squared,
                                                       T* omega) {
    T tau = 0;
#pragma unroll
    for (int m = 1; m <= M; ++m) tau += fabs(beta[0] - beta[m]);
    tau *= (T)(1.0 / M);
    const T tau2 = tau * tau;
    const T eps = (T)s.eps;
    const bool sq = SQ < 0 ? squared != 0 : SQ != 0;
    T wt[M + 1], sum = 0;
#pragma unroll
    for (int m = 0; m <= M; ++m) {
        const T den = sq ? beta[m] * beta[m] + eps : beta[m] + eps;
        wt[m] = (T)s.gam[m] * ((T)1 + tau2 * rcp(den));
        sum += wt[m];
    }
    const T inv = rcp(sum);
#pragma unroll
    for (int m = 0; m <= M; ++m) omega[m] = wt[m] * inv;
}

// The form is chosen per launch.  BRANCH: a branch on the wave-uniform flag,
// each side with the form fixed at compile time (fewer instructions, more
// code); else one copy selecting the denominator per value (fewer registers,
// which bound the occupancy of the 1D kernel).
template <class T, int M, bool BRANCH>
__device__ __forceinline__ void nonlinear_weights(const T* beta, const Scheme& s, int squared,
                                                  T* omega) {
    if (s.weights == W_LINEAR) {
#pragma unroll
        for (int m = 0; m <= M; ++m) omega[m] = (T)s.gam[m];
    } else if (!BRANCH) {
        nonlinear_weights_form<T, M, -1>(beta, s, squared, omega);
    } else if (squared) {
        nonlinear_weights_form<T, M, 1>(beta, s, squared, omega);
    } else {
        nonlinear_weights_form<T, M, 0>(beta, s, squared, omega);
    }
}

}  // namespace hweno

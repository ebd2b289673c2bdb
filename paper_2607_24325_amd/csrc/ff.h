// Compensated single-precision arithmetic for the F32_KAHAN mode: a cell
// average is held as an unevaluated sum hi + lo of two floats (about 48
// significant bits), and the cell-average update (flux differences, the
// residual and the RK combination) runs on such pairs with the error-free
// transformations two-sum (Knuth) and two-product (via FMA).  Everything else
// of the stage stays in plain FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace hweno {

// Storage of a compensated cell average (8 bytes, like a double).
struct ffs {
    float hi, lo;
    ffs() = default;
    __host__ __device__ explicit ffs(double v) : hi((float)v), lo((float)(v - (double)hi)) {}
    __host__ __device__ explicit operator double() const { return (double)hi + (double)lo; }
    __host__ __device__ explicit operator float() const { return hi + lo; }
};

__host__ __device__ inline ffs operator-(ffs a) {
    ffs r;
    r.hi = -a.hi;
    r.lo = -a.lo;
    return r;
}

// Difference of two stored averages, rounded once to float: the hi parts of
// neighbouring averages are close, so hi - hi is exact (Sterbenz) or nearly.
__device__ __forceinline__ float operator-(ffs a, ffs b) { return (a.hi - b.hi) + (a.lo - b.lo); }

// Contraction is switched off in every routine below: fused forms of these
// exact-rounding-error expressions would cancel the error terms.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
    s = a + b;
    const float bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

__device__ __forceinline__ void fast_two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
    s = a + b;
    e = b - (s - a);
}

// Compensated arithmetic value.
struct ff {
    float hi, lo;
    ff() = default;
    __device__ ff(int v) : hi((float)v), lo(0.f) {}
    __device__ ff(float v) : hi(v), lo(0.f) {}
    __device__ ff(float h, float l) : hi(h), lo(l) {}
    __device__ explicit ff(double v) : hi((float)v), lo((float)(v - (double)hi)) {}
    __device__ explicit ff(ffs s) : hi(s.hi), lo(s.lo) {}
    __device__ explicit operator float() const { return hi + lo; }
    __device__ explicit operator double() const { return (double)hi + (double)lo; }
    __device__ explicit operator ffs() const {
        ffs r;
        fast_two_sum(hi, lo, r.hi, r.lo);
        return r;
    }
};

__device__ __forceinline__ ff operator-(ff a) { return ff(-a.hi, -a.lo); }

__device__ __forceinline__ ff operator+(ff a, ff b) {
#pragma clang fp contract(off)
    float s, e;
    two_sum(a.hi, b.hi, s, e);
    e += a.lo + b.lo;
    ff r;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
}

__device__ __forceinline__ ff operator-(ff a, ff b) { return a + (-b); }

__device__ __forceinline__ ff operator*(ff a, ff b) {
#pragma clang fp contract(off)
    const float p = a.hi * b.hi;
    float e = fmaf(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    ff r;
    fast_two_sum(p, e, r.hi, r.lo);
    return r;
}

}  // namespace hweno

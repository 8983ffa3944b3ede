// Forward-mode dual numbers for the adjoint kernel: a value and its
// derivative along one parameter direction.  The geometry and Fock kernels
// are templated on their scalar types, so evaluating them on duals carries
// the chain rule through every step.
//
// The arithmetic operators are hidden friends (non-template functions found
// by argument-dependent lookup), so a plain number on either side converts to
// a constant dual; a dual of another base type never converts implicitly.
#pragma once

#include "utd_device.h"

#include <math.h>

namespace utd {

template <typename T> struct Dual {
    T v, d;
    __device__ __forceinline__ Dual() = default;
    __device__ __forceinline__ constexpr Dual(T x) : v(x), d(0) {}
    __device__ __forceinline__ constexpr Dual(T x, T dx) : v(x), d(dx) {}
    template <typename U>
    __device__ __forceinline__ explicit Dual(const Dual<U>& o) : v((T)o.v), d((T)o.d) {}

    friend __device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
    friend __device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
    friend __device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
    friend __device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
    friend __device__ __forceinline__ Dual operator/(Dual a, Dual b) {
        T q = a.v / b.v;
        return Dual(q, (a.d - q * b.d) / b.v);
    }
    friend __device__ __forceinline__ Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
    friend __device__ __forceinline__ Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
    friend __device__ __forceinline__ Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
    friend __device__ __forceinline__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
    friend __device__ __forceinline__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
    friend __device__ __forceinline__ bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
    friend __device__ __forceinline__ bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
    friend __device__ __forceinline__ bool operator==(Dual a, Dual b) { return a.v == b.v; }
    friend __device__ __forceinline__ bool operator!=(Dual a, Dual b) { return a.v != b.v; }
};

template <typename T> struct BaseOf { using type = T; };
template <typename T> struct BaseOf<Dual<T>> { using type = T; };

// value of a plain or dual scalar
__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ float val(float x) { return x; }
template <typename T> __device__ __forceinline__ T val(Dual<T> x) { return x.v; }
template <typename G> __device__ __forceinline__ d3 val3(V3<G> a) { return d3{val(a.x), val(a.y), val(a.z)}; }

// sin and cos of a moderate FP64 angle (|x| < 1e4: the geometry's angles
// stay within a few turns).  Cody-Waite reduction by pi/2 with a two-term
// constant (pi/2 = P1 + P2, P1 the double nearest pi/2, the first product
// exact through the fused multiply-add), then the Taylor series of sin and
// cos on [-pi/4, pi/4] to the x^17 / x^18 terms (truncation < 2e-19).  Short
// and register-light compared with a full-range library routine.
__device__ __forceinline__ void sincos_moderate(double x, double* s, double* c) {
    const double P1 = 1.5707963267948966192;          // double nearest pi/2
    const double P2 = 6.123233995736766036e-17;        // pi/2 - P1
    double k = rint(x * 0.63661977236758134308);       // x * 2/pi
    double r = fma(-k, P1, x);
    r = fma(-k, P2, r);
    double r2 = r * r;
    // sin r = r - r^3 (1/3! - r^2/5! + ... - r^14/17!), cos r = 1 - r^2 (1/2! - r^2/4! + ... + r^16/18!)
    double ps = -1.0 / 355687428096000.0;              // -1/17!
    ps = fma(ps, r2, 1.0 / 1307674368000.0);           //  1/15!
    ps = fma(ps, r2, -1.0 / 6227020800.0);             // -1/13!
    ps = fma(ps, r2, 1.0 / 39916800.0);                //  1/11!
    ps = fma(ps, r2, -1.0 / 362880.0);                 // -1/9!
    ps = fma(ps, r2, 1.0 / 5040.0);                    //  1/7!
    ps = fma(ps, r2, -1.0 / 120.0);                    // -1/5!
    ps = fma(ps, r2, 1.0 / 6.0);                       //  1/3!
    double sn = fma(-r * r2, ps, r);
    double pc = 1.0 / 6402373705728000.0;              //  1/18!
    pc = fma(pc, r2, -1.0 / 20922789888000.0);         // -1/16!
    pc = fma(pc, r2, 1.0 / 87178291200.0);             //  1/14!
    pc = fma(pc, r2, -1.0 / 479001600.0);              // -1/12!
    pc = fma(pc, r2, 1.0 / 3628800.0);                 //  1/10!
    pc = fma(pc, r2, -1.0 / 40320.0);                  // -1/8!
    pc = fma(pc, r2, 1.0 / 720.0);                     //  1/6!
    pc = fma(pc, r2, -1.0 / 24.0);                     // -1/4!
    pc = fma(pc, r2, 0.5);                             //  1/2!
    double cs = fma(-r2, pc, 1.0);
    int q = ((int)k) & 3;
    double so = (q & 1) ? cs : sn, co = (q & 1) ? sn : cs;
    *s = (q & 2) ? -so : so;
    *c = ((q + 1) & 2) ? -co : co;
}

// elementary functions of the geometry scalar (FP64 or dual FP64)
__device__ __forceinline__ double gsqrt(double x) { return ::sqrt(x); }
__device__ __forceinline__ double gatan2(double y, double x) { return ::atan2(y, x); }
__device__ __forceinline__ void gsincos(double x, double* s, double* c) { sincos_moderate(x, s, c); }
__device__ __forceinline__ double gfloor(double x) { return ::floor(x); }
// 1/x and 1/sqrt(x): the hardware estimate refined by two Newton steps (each
// squares the relative error), within a few ulp of the rounded quotient and
// without a division's scaling and fix-up steps.  For zero or infinite x the
// estimate itself (infinity or zero) is returned.
__device__ __forceinline__ double grcp(double x) {
    const double r0 = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r0, 1.0);
    double r = fma(r0, e, r0);
    e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    return r == r ? r : r0;
}
__device__ __forceinline__ double grsqrt(double x) {
    const double y0 = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y0, y0, 1.0);   // 1 - x y^2
    double y = fma(0.5 * y0, e, y0);
    e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    return y == y ? y : y0;
}

__device__ __forceinline__ Dual<double> gsqrt(Dual<double> x) {
    double r = ::sqrt(x.v);
    return Dual<double>(r, r > 0.0 ? x.d / (2.0 * r) : 0.0);
}
__device__ __forceinline__ Dual<double> gatan2(Dual<double> y, Dual<double> x) {
    double r2 = x.v * x.v + y.v * y.v;
    return Dual<double>(::atan2(y.v, x.v), r2 > 0.0 ? (x.v * y.d - y.v * x.d) / r2 : 0.0);
}
__device__ __forceinline__ void gsincos(Dual<double> x, Dual<double>* s, Dual<double>* c) {
    double sv, cv;
    sincos_moderate(x.v, &sv, &cv);
    *s = Dual<double>(sv, cv * x.d);
    *c = Dual<double>(cv, -sv * x.d);
}
__device__ __forceinline__ double gfloor(Dual<double> x) { return ::floor(x.v); }
__device__ __forceinline__ Dual<double> grcp(Dual<double> x) {
    const double r = grcp(x.v);
    return Dual<double>(r, -x.d * r * r);
}
__device__ __forceinline__ Dual<double> grsqrt(Dual<double> x) {
    const double y = grsqrt(x.v);
    return Dual<double>(y, -0.5 * x.d * y * y * y);
}

template <> struct RT<Dual<float>> {
    using D = Dual<float>;
    static __device__ __forceinline__ D sqrt_(D x) {
        float r = __builtin_sqrtf(x.v);
        return D(r, r > 0.0f ? x.d / (2.0f * r) : 0.0f);
    }
    static __device__ __forceinline__ D exp_(D x) {
        float e = expf(x.v);
        return D(e, e * x.d);
    }
    static __device__ __forceinline__ D cbrt_(D x) {
        float r = cbrtf(x.v);
        return D(r, r != 0.0f ? x.d / (3.0f * r * r) : 0.0f);
    }
    static __device__ __forceinline__ D rint_(D x) { return D(rintf(x.v), 0.0f); }
    static __device__ __forceinline__ D floor_(D x) { return D(floorf(x.v), 0.0f); }
    static __device__ __forceinline__ D rcp(D x) {
        float r = 1.0f / x.v;
        return D(r, -x.d * r * r);
    }
};
template <> struct RT<Dual<double>> {
    using D = Dual<double>;
    static __device__ __forceinline__ D sqrt_(D x) {
        double r = ::sqrt(x.v);
        return D(r, r > 0.0 ? x.d / (2.0 * r) : 0.0);
    }
    static __device__ __forceinline__ D exp_(D x) {
        double e = ::exp(x.v);
        return D(e, e * x.d);
    }
    static __device__ __forceinline__ D cbrt_(D x) {
        double r = ::cbrt(x.v);
        return D(r, r != 0.0 ? x.d / (3.0 * r * r) : 0.0);
    }
    static __device__ __forceinline__ D rint_(D x) { return D(::rint(x.v), 0.0); }
    static __device__ __forceinline__ D floor_(D x) { return D(::floor(x.v), 0.0); }
    static __device__ __forceinline__ D rcp(D x) {
        double r = 1.0 / x.v;
        return D(r, -x.d * r * r);
    }
};

// sin/cos of 2 pi r (revolutions) on duals
__device__ __forceinline__ void sincos_rev(Dual<float> r, Dual<float>* s, Dual<float>* c) {
    float sv, cv;
    sincos_rev(r.v, &sv, &cv);
    const float w = 6.28318530717958647692f;
    *s = Dual<float>(sv, w * cv * r.d);
    *c = Dual<float>(cv, -w * sv * r.d);
}
__device__ __forceinline__ void sincos_rev(Dual<double> r, Dual<double>* s, Dual<double>* c) {
    double sv, cv;
    sincos_rev(r.v, &sv, &cv);
    const double w = kTwoPi;
    *s = Dual<double>(sv, w * cv * r.d);
    *c = Dual<double>(cv, -w * sv * r.d);
}

}  // namespace utd

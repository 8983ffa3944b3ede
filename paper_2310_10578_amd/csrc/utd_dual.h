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

// elementary functions of the geometry scalar (FP64 or dual FP64)
__device__ __forceinline__ double gsqrt(double x) { return ::sqrt(x); }
__device__ __forceinline__ double gatan2(double y, double x) { return ::atan2(y, x); }
__device__ __forceinline__ void gsincos(double x, double* s, double* c) { ::sincos(x, s, c); }
__device__ __forceinline__ double gfloor(double x) { return ::floor(x); }

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
    ::sincos(x.v, &sv, &cv);
    *s = Dual<double>(sv, cv * x.d);
    *c = Dual<double>(cv, -sv * x.d);
}
__device__ __forceinline__ double gfloor(Dual<double> x) { return ::floor(x.v); }

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

// Device-side building blocks of the smooth-surface UTD field evaluation
// (gfx950).  Included by utd_kernels.hip only.
//
// Notation follows the paper (Sec. II-B, Eqs. (1)-(4)) and the off-surface
// UTD it cites (Pathak, Burnside and Marhefka 1980): source T, receiver R,
// attachment Q1, detachment Q2, reflection point Q_R, arc length t, incident
// and shed lengths s^i, s^d, Fock parameter m = (k rho_g / 2)^{1/3},
// xi = int m / rho_g dt, transition argument X, distance parameter L.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace utd {

constexpr double kC0 = 299792458.0;
constexpr double kTwoPi = 6.283185307179586476925287;
constexpr double kPi = 3.141592653589793238462643;
constexpr double kInvTwoPi = 0.1591549430918953357688837;

// mask bits per (body, receiver): creeping path (side, ell) valid and visible
// -> bit 2*ell + (side < 0); reflection -> bit 6; axial caustic drop -> bit 7
constexpr int kBitRefl = 6;
constexpr int kBitCaustic = 7;
constexpr uint8_t kFlagInside = 1, kFlagCaustic = 2, kFlagLos = 4, kFlagTxInside = 8;
// invalid inputs found on the device: a non-finite receiver (that receiver
// gets E = 0), an invalid body of the call or frame (every receiver gets
// E = 0), an invalid frequency (E = 0 at that frequency, every receiver
// flagged)
constexpr uint8_t kFlagInvalidRx = 16, kFlagBadBody = 32, kFlagBadFreq = 64;
// receivers whose field is zero at every frequency
constexpr uint8_t kFlagDead = kFlagInside | kFlagTxInside | kFlagInvalidRx | kFlagBadBody;
// bits of the device-wide input status word (utd_input_status)
constexpr unsigned kBadRx = 1u, kBadBody = 2u, kBadFreq = 4u;

struct LaunchParams {
    double T[3];          // source position
    double p[3];          // dipole
    double amp;           // amplitude
    int n_sph, n_cyl;
    int64_t n_rx;
    int n_f;
    int l_enc, bodies_occlude, lit_branch;
    double caustic_guard;
    int broot;            // root node of the boundary-triangle tree (-1: none)
    float blo[3], bhi[3]; // scene bounding box (the boundary triangles lie in its faces)
};

// Per-body quantities that depend only on the source (computed once per call).
template <typename G> struct BodyPrepT {
    G c[3];           // sphere centre / cylinder axis point (cx, cy, 0)
    G a;              // radius
    double z0, h;     // cylinder lateral surface z0 .. z0 + h
    G eT[3];          // sphere: unit (T - C); cylinder: unit (T - c) in xy
    G dT;             // sphere: |T - C|; cylinder: rho_T (distance to axis)
    G sI0;            // tangent length sqrt(dT^2 - a^2)
    G gT;             // tangent half-angle gamma_T = atan2(sI0, a)
    G aT;             // cylinder: azimuth of T about the axis
    int kind;         // 0 sphere, 1 cylinder
    int ok;           // 1 if T lies outside the body's circle/sphere
};
using BodyPrep = BodyPrepT<double>;

// Per-frequency constants (computed once per call): phase revolutions per
// metre f/c, wavenumber k, k^{1/3}, k^{1/6}, k^{-1/6}, sqrt(k) and the
// reciprocals of k^{1/3} and sqrt(k), in both precisions.
struct FreqConst {
    double rev_per_m;
    double kd, k13d, k16d, km16d, skd, ik13d, iskd;
    float kf, k13f, k16f, km16f, skf, ik13f, iskf;
    int ok;               // 0: the frequency is not finite or not > 0 (field zero)
};

// ---------------------------------------------------------------------------
// small vector helpers (plain double here; generic versions in utd_geom.h)
// ---------------------------------------------------------------------------
template <typename G> struct V3 { G x, y, z; };
using d3 = V3<double>;
__device__ __forceinline__ d3 mk(double x, double y, double z) { return d3{x, y, z}; }
template <typename G> __device__ __forceinline__ V3<G> operator+(V3<G> a, V3<G> b) { return V3<G>{a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename G> __device__ __forceinline__ V3<G> operator-(V3<G> a, V3<G> b) { return V3<G>{a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename G, typename S> __device__ __forceinline__ V3<G> operator*(S s, V3<G> a) { return V3<G>{s * a.x, s * a.y, s * a.z}; }
template <typename G> __device__ __forceinline__ G dot(V3<G> a, V3<G> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename G> __device__ __forceinline__ V3<G> cross(V3<G> a, V3<G> b) {
    return V3<G>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double norm(d3 a) { return sqrt(dot(a, a)); }

// A unit vector perpendicular to e (only used for degenerate collinear cases).
__device__ __forceinline__ d3 any_perp(d3 e) {
    d3 ref = fabs(e.x) < 0.9 ? mk(1, 0, 0) : mk(0, 1, 0);
    d3 c = cross(e, ref);
    return (1.0 / norm(c)) * c;
}

// ---------------------------------------------------------------------------
// Real-type traits: float for the FP32 path, double for the FP64 path.
// ---------------------------------------------------------------------------
template <typename R> struct RT;
template <> struct RT<float> {
    // the hardware square root (about an ulp) and the cube root from the
    // hardware base-2 logarithm and exponential (a few ulp, positive
    // arguments only): FP32 path constants, far from the FP32 tolerance
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float exp_(float x) { return expf(x); }
    static __device__ __forceinline__ float cbrt_(float x) { return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f)); }
    static __device__ __forceinline__ float rint_(float x) { return rintf(x); }
    static __device__ __forceinline__ float floor_(float x) { return floorf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
};
template <> struct RT<double> {
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
    static __device__ __forceinline__ double cbrt_(double x) { return cbrt(x); }
    static __device__ __forceinline__ double rint_(double x) { return rint(x); }
    static __device__ __forceinline__ double floor_(double x) { return floor(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
};

template <typename R> struct cplx { R re, im; };
template <typename R> __device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return cplx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// sin and cos of 2 pi r for r in [-1/2, 1] (revolutions).  FP64: the device
// library's sincospi.
// FP32: the hardware v_sin_f32 / v_cos_f32, which take their argument in
// revolutions (measured on gfx950 over [-1/2, 1/2] and over [0, 1): max abs
// error 1.25e-7, the same as a degree-9 polynomial after octant reduction).
__device__ __forceinline__ void sincos_rev(float r, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void sincos_rev(double r, double* s, double* c) { sincospi(2.0 * r, s, c); }

// e^{-j theta} for theta given in revolutions as an FP64 value, reduced to
// its fractional part in [0, 1) in FP64.
template <typename R> __device__ __forceinline__ cplx<R> phase_rev(double rev) {
    double fr = __builtin_amdgcn_fract(rev);
    R s, c;
    sincos_rev((R)fr, &s, &c);
    return cplx<R>{c, -s};
}

// e^{-j x} for a moderate real x of type R.
template <typename R> __device__ __forceinline__ cplx<R> expmj(R x) {
    R r = x * (R)kInvTwoPi;
    r = r - RT<R>::rint_(r);
    R s, c;
    sincos_rev(r, &s, &c);
    return cplx<R>{c, -s};
}

}  // namespace utd

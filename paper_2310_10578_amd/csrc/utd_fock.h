// Fock-type coefficient kernels of the off-surface UTD, evaluated from the
// piecewise polynomials of fock_tables.h.
//
// Creeping path (Eq. (4)):   T_p = -sqrt(2) m^ k^{-1/6} B_p(xi, X)   (m = m^ k^{1/3})
// Reflection     (Eq. (3)):  R_p sqrt(rho_1) = 2 sqrt(rho_1/(-xi)) Rbar_p(xi, X),
//                            Rbar_p = -e^{-j xi^3/12} B_p(xi, X)
// with B_p(xi, X) = p*_p(xi) + e^{-j pi/4} (1 - F(X)) / (2 sqrt(pi) xi)
//                 = Ptilde_p(xi) - e^{-j pi/4} F(X) / (2 sqrt(pi) xi),
// F the Kouyoumjian-Pathak transition function.  Three regimes of xi:
//   xi >= PT_HI (deep shadow):  p* from its table, 1 - F without cancellation;
//   PT_LO <= xi < PT_HI:        Ptilde from its table, F(X)/xi = sgn q F/sqrt(X);
//   xi < PT_LO (deep lit):      c = sqrt(-4/xi) e^{-j xi^3/12} p* from its table
//                               in t = (PT_LO/xi)^3.
// The regime only changes the segment index, the local variable and a few
// combining operations; the polynomial evaluation is shared.
#pragma once

#include "fock_tables.h"
#include "utd_device.h"
#include "utd_dual.h"

namespace utd {

constexpr double kInv2SqrtPi = 0.28209479177387814347;   // 1/(2 sqrt(pi))
constexpr double kRs2 = 0.70710678118654752440;          // 1/sqrt(2)

// Table geometry per precision.  Segments sit on a common index axis w
// (segment j covers [j, j + 1], local variable s = 2 (w - j) - 1):
//   regime table     [CL | PT | DS]: w = NCL t for xi < PT_LO
//                    (t = (PT_LO/xi)^3), w = NCL + RW (xi - PT_LO) beyond;
//   transition table [FA | FH]:      w = NT u / FA_HI for u < FA_HI,
//                    w = 2 NT - NT FA_HI^2 / X beyond.
template <typename T> struct TabDims;
template <> struct TabDims<float> {
    static constexpr int DEG = FT_F32_DEG, ROWS = DEG + 1;
    static constexpr int RW = FT_F32_RW, NCL = FT_F32_NCL, NPT = FT_F32_NPT, NDS = FT_F32_NDS, NT = FT_F32_NT;
};
template <> struct TabDims<double> {
    static constexpr int DEG = FT_F64_DEG, ROWS = DEG + 1;
    static constexpr int RW = FT_F64_RW, NCL = FT_F64_NCL, NPT = FT_F64_NPT, NDS = FT_F64_NDS, NT = FT_F64_NT;
};

// Pointers to the regime table ([seg][ROWS][4] = (re_s, im_s, re_h, im_h))
// and the transition table ([seg][ROWS][2] = (re, im)), in LDS (FP32) or
// global memory (FP64).
template <typename T> struct Tabs {
    const T* reg;
    const T* tf;
};

// Polynomials are evaluated in the arithmetic type R (plain or dual) from
// coefficients of the table type T.
template <typename T, typename R>
__device__ __forceinline__ void horner4(const T* seg, R s, R out[4]) {
    constexpr int D = TabDims<T>::DEG;
    const T* c = seg + 4 * D;
    R a0 = c[0], a1 = c[1], a2 = c[2], a3 = c[3];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        c -= 4;
        a0 = a0 * s + c[0];
        a1 = a1 * s + c[1];
        a2 = a2 * s + c[2];
        a3 = a3 * s + c[3];
    }
    out[0] = a0; out[1] = a1; out[2] = a2; out[3] = a3;
}

// float specialisation reading float4 rows (one 16-byte LDS read per coefficient)
template <>
__device__ __forceinline__ void horner4<float, float>(const float* seg, float s, float out[4]) {
    constexpr int D = TabDims<float>::DEG;
    const float4* c = reinterpret_cast<const float4*>(seg) + D;
    float4 a = *c;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        --c;
        float4 b = *c;
        a.x = a.x * s + b.x;
        a.y = a.y * s + b.y;
        a.z = a.z * s + b.z;
        a.w = a.w * s + b.w;
    }
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
}

template <typename T, typename R>
__device__ __forceinline__ void horner2(const T* seg, R s, R out[2]) {
    constexpr int D = TabDims<T>::DEG;
    const T* c = seg + 2 * D;
    R a0 = c[0], a1 = c[1];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        c -= 2;
        a0 = a0 * s + c[0];
        a1 = a1 * s + c[1];
    }
    out[0] = a0; out[1] = a1;
}

// Segment j = floor(w) of index-axis position w clamped to [0, wmax] (wmax
// just below the table's segment count) and the segment's local variable:
// sigma = w - j in [0, 1) for the FP32 tables, s = 2 (w - j) - 1 in [-1, 1]
// for the FP64 tables (their coefficients are stored in those variables).
__device__ __forceinline__ int seg_at(float w, float wmax, float* s) {
    w = __builtin_amdgcn_fmed3f(w, 0.0f, wmax);
    *s = __builtin_amdgcn_fractf(w);
    return (int)w;
}
__device__ __forceinline__ int seg_at(double w, double wmax, double* s) {
    w = fmin(fmax(w, 0.0), wmax);
    *s = fma(__builtin_amdgcn_fract(w), 2.0, -1.0);
    return (int)w;
}
template <typename T>
__device__ __forceinline__ int seg_at(Dual<T> w, Dual<T> wmax, Dual<T>* s) {
    constexpr bool kSigma = sizeof(T) == 4;
    T v = w.v < (T)0 ? (T)0 : (w.v > wmax.v ? wmax.v : w.v);
    int j = (int)v;
    // a clamped position does not move with the parameter
    T dv = v == w.v ? w.d : (T)0;
    *s = kSigma ? Dual<T>(v - (T)j, dv) : Dual<T>((T)2 * (v - (T)j) - (T)1, (T)2 * dv);
    return j;
}

// largest representable value below the segment count n, as the clamp
template <typename T> __host__ __device__ constexpr T below(int n) {
    return (T)n * ((T)1 - (T)(sizeof(T) == 4 ? 1.1920928955078125e-07 : 4.4408920985006262e-16));
}

// e^{z dx} for the first creeping mode z = zre + j zim (deep shadow beyond
// the table); the FP32 version takes the hardware exp2 and the revolution-
// argument sin/cos directly.
template <typename R>
__device__ __forceinline__ cplx<R> mode_factor(R dx, double zre, double zim) {
    R e = RT<R>::exp_((R)zre * dx);
    cplx<R> r = expmj<R>(-(R)zim * dx);
    return cplx<R>{e * r.re, e * r.im};
}
template <>
__device__ __forceinline__ cplx<float> mode_factor<float>(float dx, double zre, double zim) {
    constexpr double kLog2e = 1.4426950408889634074;
    float e = __builtin_amdgcn_exp2f((float)(zre * kLog2e) * dx);
    float r = (float)(-zim * kInvTwoPi) * dx;
    r -= rintf(r);
    float sn, cs;
    sincos_rev(r, &sn, &cs);
    return cplx<float>{e * cs, -e * sn};
}

// B-type kernels K_s, K_h of one path at one frequency.
//   creeping (refl = false): K = B_p(xi, X)
//   reflection (refl = true): K = Rbar_p = -e^{-j xi^3/12} B_p(xi, X)
// q = sqrt(X)/|xi| = sqrt(k L / 2)/m enters explicitly (finite at xi = 0), as
// qc = -kC2E4 q, and 1/xi also as xc = kC2E4/xi: per path the constant
// factor folds into the path's own constant.
// Written without data-dependent branches: the regime and the transition
// range only select the segment, the local variable and a few operands, so a
// wavefront whose lanes sit in different regimes stays converged.
// MODE selects a specialisation for wavefronts whose lanes all hold the same
// kind of path: kCreep (creeping paths: xi >= 0, regimes 0/1, K = B_p), kRefl
// (reflections: xi <= 0, regimes 1/2, K = Rbar_p) or kAny (mixed lanes).
enum { kAny = 0, kCreep = 1, kRefl = 2 };
// e^{-j pi/4}/(2 sqrt pi) = kC2E4 (1 - j)
constexpr double kC2E4 = kInv2SqrtPi * kRs2;

template <typename R> struct FockArgs {
    R xi;    // Fock parameter
    R u;     // sqrt(X), X the transition-function argument
    R iu;    // 1/u (any value when u < FA_HI)
    R ixi;   // 1/xi (0 when xi == 0)
    R h;     // sqrt(-xi)/2 (deep lit; 0 otherwise)
    R qc;    // -kC2E4 q, q = sqrt(X)/|xi| (finite at xi = 0)
    R xc;    // kC2E4 / xi
};

template <typename R, int MODE = kAny>
__device__ __forceinline__ void fock_kernel(const Tabs<typename BaseOf<R>::type>& tb, const FockArgs<R>& A, bool refl,
                                            cplx<R>* Ks, cplx<R>* Kh) {
    using T = typename BaseOf<R>::type;
    using D = TabDims<T>;
    const R xi = A.xi, u = A.u, ixi = A.ixi;

    // --- transition function: A(u) for u < FA_HI, H(1/X) beyond -------------
    // The segment decides which of the two is read, so the two sides of the
    // junction stay consistent under rounding.
    const R iu = A.iu, iX = iu * iu;
    R wt = u >= (R)FT_FA_HI ? (R)(2 * D::NT) - (R)(D::NT * FT_FA_HI * FT_FA_HI) * iX
                            : u * (R)(D::NT / FT_FA_HI);
    R st;
    const int tseg = seg_at(wt, (R)below<T>(2 * D::NT), &st);
    const bool big = tseg >= D::NT;
    R v[2];
    horner2<T, R>(tb.tf + __umul24((unsigned)tseg, 2 * D::ROWS), st, v);
    // the table holds v = G = F/sqrt(X) below FA_HI and v = -H = (1 - F) X
    // above; G and 1 - F follow as A0 + A1 v (below: G = v, 1 - F = 1 - u v;
    // above: G = (1 - iX v) iu, 1 - F = iX v) with real A0, A1 chosen below

    // --- regime table ------------------------------------------------------
    // creeping paths have xi >= 0 (regimes 0, 1), reflections xi <= 0 (1, 2);
    // the regime follows from the segment
    const R w_xi = xi * (R)D::RW + (R)(D::NCL - FT_PT_LO * D::RW);
    R w;
    if (MODE == kCreep) {
        w = w_xi;
    } else {
        R r3 = (R)FT_PT_LO * ixi;
        w = xi >= (R)FT_PT_LO ? w_xi : r3 * r3 * r3 * (R)D::NCL;
    }
    R s;
    const int seg = seg_at(w, (R)below<T>(D::NCL + D::NPT + D::NDS), &s);
    const int regime = (MODE != kRefl && seg >= D::NCL + D::NPT) ? 0 : ((MODE == kCreep || seg >= D::NCL) ? 1 : 2);
    R w4[4];
    horner4<T, R>(tb.reg + __umul24((unsigned)seg, 4 * D::ROWS), s, w4);
    cplx<R> ps{w4[0], w4[1]}, ph{w4[2], w4[3]};
    if (MODE != kRefl && xi > (R)FT_DS_HI) {
        // past the table only the first creeping mode survives:
        // scale the end value by e^{z1 (xi - DS_HI)} (rare)
        R dx = xi - (R)FT_DS_HI;
        ps = cmul(ps, mode_factor<R>(dx, FT_Z1S_RE, FT_Z1S_IM));
        ph = cmul(ph, mode_factor<R>(dx, FT_Z1H_RE, FT_Z1H_IM));
    }

    // --- combine ------------------------------------------------------------
    // CW = e^{-j pi/4} coef W:  regime 1: coef = -sgn q/(2 sqrt pi), W = G
    //                          regimes 0, 2: coef = 1/(2 sqrt(pi) xi), W = 1 - F
    const bool r1 = regime == 1;
    const R A1 = big ? (r1 ? -(iX * iu) : iX) : (r1 ? (R)1 : -u);
    const R A0 = big ? (r1 ? iu : (R)0) : (r1 ? (R)0 : (R)1);
    const cplx<R> W{A0 + A1 * v[0], A1 * v[1]};
    if (MODE == kCreep) {
        // sgn(xi) = +1 for creeping paths (xi >= 0); K = P + CW
        R f = r1 ? A.qc : A.xc;
        cplx<R> CW{f * (W.re + W.im), f * (W.im - W.re)};
        *Ks = cplx<R>{ps.re + CW.re, ps.im + CW.im};
        *Kh = cplx<R>{ph.re + CW.re, ph.im + CW.im};
        return;
    }
    cplx<R> e = expmj<R>(xi * xi * xi * (R)(1.0 / 12));
    if (MODE == kRefl) {
        // sgn = -1 on the lit side (xi <= 0): coef = q/(2 sqrt pi) in regime 1;
        // K = -(alpha P + e CW), alpha = e (regime 1) or sqrt(-xi)/2 (regime 2)
        R f = r1 ? -A.qc : A.xc;
        cplx<R> CW{f * (W.re + W.im), f * (W.im - W.re)};
        cplx<R> eCW = cmul(e, CW);
        const bool r2 = regime == 2;
        const cplx<R> al{r2 ? A.h : e.re, r2 ? (R)0 : e.im};
        cplx<R> as = cmul(al, ps), ah = cmul(al, ph);
        *Ks = cplx<R>{-(as.re + eCW.re), -(as.im + eCW.im)};
        *Kh = cplx<R>{-(ah.re + eCW.re), -(ah.im + eCW.im)};
        return;
    }
    R sg = refl ? (xi > (R)0 ? (R)1 : (R)-1) : (xi < (R)0 ? (R)-1 : (R)1);
    R f = r1 ? sg * A.qc : A.xc;
    cplx<R> CW{f * (W.re + W.im), f * (W.im - W.re)};
    // creeping: K = P + CW
    // reflection / deep lit: K = -(alpha P + e CW), e = e^{-j xi^3/12},
    //   alpha = e (regimes 0, 1) or sqrt(-xi)/2 (regime 2, P = c)
    bool lit = refl || regime == 2;
    cplx<R> alpha = regime == 2 ? cplx<R>{A.h, (R)0} : e;
    cplx<R> eCW = cmul(e, CW);
    cplx<R> as = cmul(alpha, ps), ah = cmul(alpha, ph);
    Ks->re = lit ? -(as.re + eCW.re) : ps.re + CW.re;
    Ks->im = lit ? -(as.im + eCW.im) : ps.im + CW.im;
    Kh->re = lit ? -(ah.re + eCW.re) : ph.re + CW.re;
    Kh->im = lit ? -(ah.im + eCW.im) : ph.im + CW.im;
}

}  // namespace utd

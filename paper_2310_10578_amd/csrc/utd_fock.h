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

// Table geometry shared by both precisions (segment counts differ).
template <typename R> struct TabDims;
// ROWS: coefficient rows stored per segment (DEG + 1, padded to a power of
// two for the LDS copy of the FP32 tables so the segment offset is a shift).
template <> struct TabDims<float> {
    static constexpr int DEG = FT_F32_PT_DEG;
    static constexpr int ROWS = 8;
    static constexpr int NPT = FT_F32_PT_NSEG, NDS = FT_F32_DS_NSEG, NCL = FT_F32_CL_NSEG;
    static constexpr int NFA = FT_F32_FA_NSEG, NFH = FT_F32_FH_NSEG;
    static_assert(DEG + 1 <= ROWS, "row padding");
};
template <> struct TabDims<double> {
    static constexpr int DEG = FT_F64_PT_DEG;
    static constexpr int ROWS = FT_F64_PT_DEG + 1;
    static constexpr int NPT = FT_F64_PT_NSEG, NDS = FT_F64_DS_NSEG, NCL = FT_F64_CL_NSEG;
    static constexpr int NFA = FT_F64_FA_NSEG, NFH = FT_F64_FH_NSEG;
};

// Pointers to the regime tables ([seg][ROWS][4] = (re_s, im_s, re_h, im_h))
// and the transition tables ([seg][ROWS][2] = (re, im)), in LDS (FP32) or
// global memory (FP64).
template <typename T> struct Tabs {
    const T* reg;   // PT segments, then DS, then CL
    const T* tf;    // FA segments, then FH
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

// Locate x in [lo, hi] split into n equal segments: index and s in [-1, 1].
template <typename R>
__device__ __forceinline__ int locate(R x, R lo, R inv_w, int n, R* s) {
    R u = (x - lo) * inv_w;
    int i = (int)val(RT<R>::floor_(u));
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    *s = (R)2 * (u - (R)i) - (R)1;
    return i;
}

// B-type kernels K_s, K_h of one path at one frequency.
//   creeping (refl = false): K = B_p(xi, X)
//   reflection (refl = true): K = Rbar_p = -e^{-j xi^3/12} B_p(xi, X)
// q = sqrt(X)/|xi| = sqrt(k L / 2)/m is passed explicitly (finite at xi = 0).
// Written without data-dependent branches: the regime and the transition
// range only select the segment, the local variable and a few operands, so a
// wavefront whose lanes sit in different regimes stays converged.
// MODE selects a specialisation for wavefronts whose lanes all hold the same
// kind of path: kCreep (creeping paths: xi >= 0, regimes 0/1, K = B_p), kRefl
// (reflections: xi <= 0, regimes 1/2, K = Rbar_p) or kAny (mixed lanes).
enum { kAny = 0, kCreep = 1, kRefl = 2 };
template <typename R> struct FockArgs {
    R xi;    // Fock parameter
    R u;     // sqrt(X), X the transition-function argument
    R q;     // sqrt(X)/|xi|
    R ixi;   // 1/xi (0 when xi == 0)
    R h;     // sqrt(-xi)/2 (deep lit; 0 otherwise)
};

template <typename R, int MODE = kAny>
__device__ __forceinline__ void fock_kernel(const Tabs<typename BaseOf<R>::type>& tb, const FockArgs<R>& A, bool refl,
                                            cplx<R>* Ks, cplx<R>* Kh) {
    using T = typename BaseOf<R>::type;
    using D = TabDims<T>;
    const R e4 = (R)kRs2;                     // e^{-j pi/4} = e4 (1 - j)
    const R c2 = (R)kInv2SqrtPi;
    const R xi = A.xi, u = A.u, q = A.q, ixi = A.ixi;

    // --- transition function: A(u) for u <= FA_HI, H(1/X) beyond -----------
    bool big = u > (R)FT_FA_HI;
    R iu = RT<R>::rcp(big ? u : (R)1);
    R iX = iu * iu;
    R targ = big ? iX : u;
    R invw = big ? (R)(D::NFH * FT_FA_HI * FT_FA_HI) : (R)(D::NFA / FT_FA_HI);
    int nseg = big ? D::NFH : D::NFA;
    R st;
    int tseg = (big ? D::NFA : 0) + locate<R>(targ, (R)0, invw, nseg, &st);
    R v[2];
    horner2<T, R>(tb.tf + tseg * 2 * D::ROWS, st, v);
    // small u: G = F/sqrt(X) = 2j A, F = u G; large u: 1 - F = -H/X, G = F/u
    R omr = -iX * v[0], omi = -iX * v[1];
    cplx<R> G, omF;
    G.re = big ? ((R)1 - omr) * iu : (R)-2 * v[1];
    G.im = big ? -omi * iu : (R)2 * v[0];
    omF.re = big ? omr : (R)1 - u * G.re;
    omF.im = big ? omi : -u * G.im;

    // --- regime table ------------------------------------------------------
    // creeping paths have xi >= 0 (regimes 0, 1), reflections xi <= 0 (1, 2)
    int regime = (MODE != kRefl && xi >= (R)FT_PT_HI) ? 0 : ((MODE == kCreep || xi >= (R)FT_PT_LO) ? 1 : 2);
    R s;
    int seg;
    if (MODE == kCreep) {
        // both regimes read xi itself, clamped to the deep-shadow table's end
        R arg = xi < (R)FT_DS_HI ? xi : (R)FT_DS_HI;
        bool r0 = regime == 0;
        seg = (r0 ? D::NPT : 0) +
              locate<R>(arg, r0 ? (R)FT_PT_HI : (R)FT_PT_LO,
                        r0 ? (R)(D::NDS / (FT_DS_HI - FT_PT_HI)) : (R)(D::NPT / (FT_PT_HI - FT_PT_LO)),
                        r0 ? D::NDS : D::NPT, &s);
    } else if (MODE == kRefl) {
        R r3 = (R)FT_PT_LO * ixi;
        bool r1 = regime == 1;
        seg = (r1 ? 0 : D::NPT + D::NDS) +
              locate<R>(r1 ? xi : r3 * r3 * r3, r1 ? (R)FT_PT_LO : (R)0,
                        r1 ? (R)(D::NPT / (FT_PT_HI - FT_PT_LO)) : (R)D::NCL, r1 ? D::NPT : D::NCL, &s);
    } else {
        R r3 = (R)FT_PT_LO * ixi;
        R arg = regime == 0 ? (xi < (R)FT_DS_HI ? xi : (R)FT_DS_HI) : (regime == 1 ? xi : r3 * r3 * r3);
        R rlo = regime == 0 ? (R)FT_PT_HI : (regime == 1 ? (R)FT_PT_LO : (R)0);
        R rinv = regime == 0 ? (R)(D::NDS / (FT_DS_HI - FT_PT_HI))
                             : (regime == 1 ? (R)(D::NPT / (FT_PT_HI - FT_PT_LO)) : (R)D::NCL);
        int rn = regime == 0 ? D::NDS : (regime == 1 ? D::NPT : D::NCL);
        int rbase = regime == 0 ? D::NPT : (regime == 1 ? 0 : D::NPT + D::NDS);
        seg = rbase + locate<R>(arg, rlo, rinv, rn, &s);
    }
    R w4[4];
    horner4<T, R>(tb.reg + seg * 4 * D::ROWS, s, w4);
    cplx<R> ps{w4[0], w4[1]}, ph{w4[2], w4[3]};
    if (MODE != kRefl && regime == 0 && xi > (R)FT_DS_HI) {
        // past the table only the first creeping mode survives:
        // scale the end value by e^{z1 (xi - DS_HI)} (rare)
        R dx = xi - (R)FT_DS_HI;
        R es = RT<R>::exp_((R)FT_Z1S_RE * dx), eh = RT<R>::exp_((R)FT_Z1H_RE * dx);
        cplx<R> rs = expmj<R>(-(R)FT_Z1S_IM * dx), rh = expmj<R>(-(R)FT_Z1H_IM * dx);
        ps = cmul(ps, cplx<R>{es * rs.re, es * rs.im});
        ph = cmul(ph, cplx<R>{eh * rh.re, eh * rh.im});
    }

    // --- combine ------------------------------------------------------------
    // CW = e^{-j pi/4} coef W:  regime 1: coef = -sgn q/(2 sqrt pi), W = G
    //                          regimes 0, 2: coef = 1/(2 sqrt(pi) xi), W = 1 - F
    cplx<R> W = regime == 1 ? G : omF;
    if (MODE == kCreep) {
        // sgn(xi) = +1 for creeping paths (xi >= 0); K = P + CW
        R f = (regime == 1 ? -q * c2 : c2 * ixi) * e4;
        cplx<R> CW{f * (W.re + W.im), f * (W.im - W.re)};
        *Ks = cplx<R>{ps.re + CW.re, ps.im + CW.im};
        *Kh = cplx<R>{ph.re + CW.re, ph.im + CW.im};
        return;
    }
    cplx<R> e = expmj<R>(xi * xi * xi * (R)(1.0 / 12));
    if (MODE == kRefl) {
        // sgn = -1 on the lit side (xi <= 0): coef = q/(2 sqrt pi) in regime 1;
        // K = -(alpha P + e CW), alpha = e (regime 1) or sqrt(-xi)/2 (regime 2)
        R f = (regime == 1 ? q * c2 : c2 * ixi) * e4;
        cplx<R> CW{f * (W.re + W.im), f * (W.im - W.re)};
        cplx<R> eCW = cmul(e, CW);
        bool r2 = regime == 2;
        cplx<R> as = cmul(e, ps), ah = cmul(e, ph);
        Ks->re = -((r2 ? A.h * ps.re : as.re) + eCW.re);
        Ks->im = -((r2 ? A.h * ps.im : as.im) + eCW.im);
        Kh->re = -((r2 ? A.h * ph.re : ah.re) + eCW.re);
        Kh->im = -((r2 ? A.h * ph.im : ah.im) + eCW.im);
        return;
    }
    R sg = refl ? (xi > (R)0 ? (R)1 : (R)-1) : (xi < (R)0 ? (R)-1 : (R)1);
    R coef = regime == 1 ? -sg * q * c2 : c2 * ixi;
    R f = coef * e4;
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

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

namespace utd {

constexpr double kInv2SqrtPi = 0.28209479177387814347;   // 1/(2 sqrt(pi))
constexpr double kRs2 = 0.70710678118654752440;          // 1/sqrt(2)

// Table geometry shared by both precisions (segment counts differ).
template <typename R> struct TabDims;
template <> struct TabDims<float> {
    static constexpr int DEG = FT_F32_PT_DEG;
    static constexpr int NPT = FT_F32_PT_NSEG, NDS = FT_F32_DS_NSEG, NCL = FT_F32_CL_NSEG;
    static constexpr int NFA = FT_F32_FA_NSEG, NFH = FT_F32_FH_NSEG;
};
template <> struct TabDims<double> {
    static constexpr int DEG = FT_F64_PT_DEG;
    static constexpr int NPT = FT_F64_PT_NSEG, NDS = FT_F64_DS_NSEG, NCL = FT_F64_CL_NSEG;
    static constexpr int NFA = FT_F64_FA_NSEG, NFH = FT_F64_FH_NSEG;
};

// Pointers to the regime tables ([seg][DEG+1][4] = (re_s, im_s, re_h, im_h))
// and the transition tables ([seg][DEG+1][2] = (re, im)), in LDS (FP32) or
// global memory (FP64).
template <typename R> struct Tabs {
    const R* reg;   // PT segments, then DS, then CL
    const R* tf;    // FA segments, then FH
};

template <typename R>
__device__ __forceinline__ void horner4(const R* seg, R s, R out[4]) {
    constexpr int D = TabDims<R>::DEG;
    const R* c = seg + 4 * D;
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
__device__ __forceinline__ void horner4<float>(const float* seg, float s, float out[4]) {
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

template <typename R>
__device__ __forceinline__ void horner2(const R* seg, R s, R out[2]) {
    constexpr int D = TabDims<R>::DEG;
    const R* c = seg + 2 * D;
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
    int i = (int)RT<R>::floor_(u);
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    *s = (R)2 * (u - (R)i) - (R)1;
    return i;
}

// Transition function: F(X), F(X)/sqrt(X) and 1 - F(X), u = sqrt(X).
template <typename R>
__device__ __forceinline__ void transition(const Tabs<R>& tb, R X, R u, cplx<R>* F, cplx<R>* G, cplx<R>* omF) {
    using D = TabDims<R>;
    R v[2], s;
    if (u <= (R)FT_FA_HI) {
        int i = locate<R>(u, (R)0, (R)D::NFA / (R)FT_FA_HI, D::NFA, &s);
        horner2<R>(tb.tf + i * 2 * (D::DEG + 1), s, v);       // A(u)
        *G = cplx<R>{-2 * v[1], 2 * v[0]};                     // 2j A
        *F = cplx<R>{-2 * u * v[1], 2 * u * v[0]};             // 2j u A
        *omF = cplx<R>{(R)1 - F->re, -F->im};
    } else {
        R iv = RT<R>::rcp(X);
        int i = locate<R>(iv, (R)0, (R)D::NFH * (R)(FT_FA_HI * FT_FA_HI), D::NFH, &s);
        horner2<R>(tb.tf + (D::NFA + i) * 2 * (D::DEG + 1), s, v);   // H(v) = (F - 1) X
        *omF = cplx<R>{-iv * v[0], -iv * v[1]};
        *F = cplx<R>{(R)1 - omF->re, -omF->im};
        R iu = RT<R>::rcp(u);
        *G = cplx<R>{F->re * iu, F->im * iu};
    }
}

// B-type kernels K_s, K_h of one path at one frequency.
//   creeping (refl = false): K = B_p(xi, X)
//   reflection (refl = true): K = Rbar_p = -e^{-j xi^3/12} B_p(xi, X)
// q = sqrt(X)/|xi| = sqrt(k L / 2)/m is passed explicitly (finite at xi = 0).
template <typename R>
__device__ __forceinline__ void fock_kernel(const Tabs<R>& tb, R xi, R X, R q, bool refl,
                                            cplx<R>* Ks, cplx<R>* Kh) {
    using D = TabDims<R>;
    const R e4 = (R)kRs2;                     // e^{-j pi/4} = e4 (1 - j)
    R u = RT<R>::sqrt_(X);
    cplx<R> F, G, omF;
    transition<R>(tb, X, u, &F, &G, &omF);

    // regime: segment and local variable in the concatenated regime table
    int seg;
    R s;
    int regime;
    if (xi >= (R)FT_PT_HI) {
        regime = 0;
        R x = xi < (R)FT_DS_HI ? xi : (R)FT_DS_HI;
        seg = D::NPT + locate<R>(x, (R)FT_PT_HI, (R)D::NDS / (R)(FT_DS_HI - FT_PT_HI), D::NDS, &s);
    } else if (xi >= (R)FT_PT_LO) {
        regime = 1;
        seg = locate<R>(xi, (R)FT_PT_LO, (R)D::NPT / (R)(FT_PT_HI - FT_PT_LO), D::NPT, &s);
    } else {
        regime = 2;
        R r = (R)FT_PT_LO * RT<R>::rcp(xi);
        R t = r * r * r;
        seg = D::NPT + D::NDS + locate<R>(t, (R)0, (R)D::NCL, D::NCL, &s);
    }
    R v[4];
    horner4<R>(tb.reg + seg * 4 * (D::DEG + 1), s, v);
    cplx<R> ps{v[0], v[1]}, ph{v[2], v[3]};

    if (regime == 0) {
        // p* + e^{-j pi/4} (1 - F) / (2 sqrt(pi) xi); beyond DS_HI only the
        // first mode survives and the last segment's value stands in for it
        R f = (R)kInv2SqrtPi * e4 * RT<R>::rcp(xi);
        cplx<R> c0{f * (omF.re + omF.im), f * (omF.im - omF.re)};
        *Ks = cplx<R>{ps.re + c0.re, ps.im + c0.im};
        *Kh = cplx<R>{ph.re + c0.re, ph.im + c0.im};
        if (xi > (R)FT_DS_HI) {
            // scale by the first-mode decay e^{z1 (xi - DS_HI)}
            R dx = xi - (R)FT_DS_HI;
            R es = RT<R>::exp_((R)FT_Z1S_RE * dx), eh = RT<R>::exp_((R)FT_Z1H_RE * dx);
            cplx<R> rs = expmj<R>(-(R)FT_Z1S_IM * dx), rh = expmj<R>(-(R)FT_Z1H_IM * dx);
            cplx<R> ks = cmul(ps, cplx<R>{es * rs.re, es * rs.im});
            cplx<R> kh = cmul(ph, cplx<R>{eh * rh.re, eh * rh.im});
            *Ks = cplx<R>{ks.re + c0.re, ks.im + c0.im};
            *Kh = cplx<R>{kh.re + c0.re, kh.im + c0.im};
        }
        if (refl) {
            cplx<R> e = expmj<R>(xi * xi * xi * (R)(1.0 / 12));
            cplx<R> a = cmul(e, *Ks), b = cmul(e, *Kh);
            *Ks = cplx<R>{-a.re, -a.im};
            *Kh = cplx<R>{-b.re, -b.im};
        }
    } else if (regime == 1) {
        // Ptilde - sgn e^{-j pi/4} q F/sqrt(X) / (2 sqrt(pi))
        R sg = refl ? (xi > (R)0 ? (R)1 : (R)-1) : (xi < (R)0 ? (R)-1 : (R)1);
        R f = sg * q * (R)kInv2SqrtPi * e4;
        cplx<R> c0{f * (G.re + G.im), f * (G.im - G.re)};
        cplx<R> bs{ps.re - c0.re, ps.im - c0.im}, bh{ph.re - c0.re, ph.im - c0.im};
        if (refl) {
            cplx<R> e = expmj<R>(xi * xi * xi * (R)(1.0 / 12));
            cplx<R> a = cmul(e, bs), b = cmul(e, bh);
            *Ks = cplx<R>{-a.re, -a.im};
            *Kh = cplx<R>{-b.re, -b.im};
        } else {
            *Ks = bs;
            *Kh = bh;
        }
    } else {
        // -c sqrt(-xi)/2 - e^{-j xi^3/12} e^{-j pi/4} (1 - F)/(2 sqrt(pi) xi)
        R h = (R)0.5 * RT<R>::sqrt_(-xi);
        R f = (R)kInv2SqrtPi * e4 * RT<R>::rcp(xi);
        cplx<R> c0{f * (omF.re + omF.im), f * (omF.im - omF.re)};
        cplx<R> e = expmj<R>(xi * xi * xi * (R)(1.0 / 12));
        cplx<R> corr = cmul(e, c0);
        *Ks = cplx<R>{-ps.re * h - corr.re, -ps.im * h - corr.im};
        *Kh = cplx<R>{-ph.re * h - corr.re, -ph.im * h - corr.im};
    }
}

}  // namespace utd

// Ray geometry of the smooth-surface UTD paths on spheres and vertical
// cylinders (device code).
//
// Creeping path (Eq. (4), Sec. III-B): tangent from the source T to the
// attachment point Q1, surface geodesic Q1 -> Q2 of length t, tangent from
// the detachment point Q2 to the receiver R.  Reflection (Eq. (3)): the
// specular point Q_R on the arc seen from both T and R.
//
// Precision: everything that enters the phase k (s^i + t + s^d) -- distances,
// tangent lengths and the arc angle phi -- is FP64.  Angles come from one
// FP64 atan2 per (receiver, body): the arcs of the two sides add up to a
// known total, and the cosines/sines of the detachment angles are algebraic
// in the distances.  Frames, spreading and Fock arguments are computed in
// the field precision R.  The reflection point is solved once (FP64
// safeguarded Newton) by the visibility pass and its angle is reused.
//
// Every function is templated on the geometry scalar G (double, or a dual
// number for the adjoint) and the field scalar R; the forward kernels
// instantiate G = double.
#pragma once

#include "utd_device.h"
#include "utd_dual.h"


namespace utd {

// Everything the frequency loop needs about one path.  With m = mhat k^{1/3},
// xi = m phi_e (phi_e = t/rho_g, or -2 cos th_i for a reflection) and
// X = k L phi_e^2 / 2, the per-frequency Fock arguments are
//   xi = k^{1/3} xh,  sqrt(X) = k^{1/2} uh,  q = k^{1/6} qhat,
//   1/xi = k^{-1/3} ixh,  sqrt(-xi) = k^{1/6} sxh,
// and the contribution is
//   e^{-j 2pi rev} k^{-1/6} (K_s v_s + K_h v_h),  rev = (f/c) s_tot - nc/4,
// where v_s, v_h are the output polarisation vectors at R scaled by the
// incident projection, the spreading and the constant prefactor.
template <typename R, typename G = double> struct PathEvalT {
    G s_tot;          // total path length s^i + t + s^d (or s^i + s^r)
    int nc;           // caustics passed (each +pi/2)
    int refl;
    R xh, uh, qhat, ixh, sxh, iuh;
    R vs[3], vh[3];   // amplitude-weighted polarisation vectors
};
template <typename R> using PathEval = PathEvalT<R, double>;

template <typename G> __device__ __forceinline__ V3<G> v3(const G c[3]) { return V3<G>{c[0], c[1], c[2]}; }
template <typename G> __device__ __forceinline__ G gnorm(V3<G> a) { return gsqrt(dot(a, a)); }

// Fill the Fock-argument constants from mhat, phi_e and L (= L^d or L^r).
template <typename R, typename G>
__device__ __forceinline__ void set_fock_consts(PathEvalT<R, G>* pe, R mhat, R phi_e, R Ld) {
    R xh = mhat * phi_e;
    R sl = RT<R>::sqrt_((R)0.5 * Ld);
    pe->xh = xh;
    pe->uh = sl * (phi_e < (R)0 ? -phi_e : phi_e);
    pe->qhat = sl * RT<R>::rcp(mhat);
    pe->ixh = xh != (R)0 ? RT<R>::rcp(xh) : (R)0;
    pe->sxh = RT<R>::sqrt_(xh < (R)0 ? -xh : (R)0);
    pe->iuh = pe->uh > (R)0 ? RT<R>::rcp(pe->uh) : (R)0;
}

// Points of a path (for the visibility tests).
struct PathPts {
    d3 P0, P1;        // first leg  T -> Q1 (or Q_R)
    d3 P2, P3;        // second leg Q2 (or Q_R) -> R
};

// Source-dependent constants of a sphere (centre C, radius a) and of a
// vertical cylinder (axis through (cx, cy), lateral surface z0 .. z0 + h).
template <typename G>
__device__ __forceinline__ BodyPrepT<G> prep_sphere(V3<G> T, V3<G> C, G a) {
    BodyPrepT<G> p;
    p.kind = 0;
    p.c[0] = C.x; p.c[1] = C.y; p.c[2] = C.z;
    p.a = a;
    p.z0 = 0; p.h = 0;
    V3<G> v = T - C;
    p.dT = gnorm(v);
    G idT = grcp(p.dT);
    p.eT[0] = v.x * idT; p.eT[1] = v.y * idT; p.eT[2] = v.z * idT;
    p.ok = p.dT > p.a;
    p.sI0 = p.ok ? gsqrt((p.dT - p.a) * (p.dT + p.a)) : G(0.0);
    p.gT = gatan2(p.sI0, p.a);
    p.aT = G(0.0);
    return p;
}

template <typename G>
__device__ __forceinline__ BodyPrepT<G> prep_cylinder(V3<G> T, G cx, G cy, double z0, double h, G a) {
    BodyPrepT<G> p;
    p.kind = 1;
    p.c[0] = cx; p.c[1] = cy; p.c[2] = G(0.0);
    p.z0 = z0; p.h = h; p.a = a;
    G tx = T.x - cx, ty = T.y - cy;
    p.dT = gsqrt(tx * tx + ty * ty);
    const G idT = grcp(p.dT);
    p.eT[0] = tx * idT; p.eT[1] = ty * idT; p.eT[2] = G(0.0);
    p.ok = p.dT > p.a;
    p.sI0 = p.ok ? gsqrt((p.dT - p.a) * (p.dT + p.a)) : G(0.0);
    p.gT = gatan2(p.sI0, p.a);
    p.aT = gatan2(ty, tx);
    return p;
}

// A body whose parameters are not finite, or whose radius is not > 0 (or a
// cylinder height < 0), is invalid: it carries no path, and every receiver
// of the call is flagged (kFlagBadBody) with a zero field.
__device__ __forceinline__ bool body_params_bad(const float* sph, int n_sph, const float* cyl, int b) {
    if (b < n_sph) {
        const float* s = sph + 4 * b;
        return !(isfinite(s[0]) && isfinite(s[1]) && isfinite(s[2]) && isfinite(s[3]) && s[3] > 0.0f);
    }
    const float* c = cyl + 5 * (b - n_sph);
    return !(isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]) && isfinite(c[3]) && isfinite(c[4]) &&
             c[3] >= 0.0f && c[4] > 0.0f);
}

__device__ __forceinline__ BodyPrep body_prep(const double T[3], const float* sph, int n_sph, const float* cyl,
                                              int b) {
    d3 t = mk(T[0], T[1], T[2]);
    BodyPrep p;
    if (b < n_sph) {
        const float* s = sph + 4 * b;
        p = prep_sphere<double>(t, mk(s[0], s[1], s[2]), (double)s[3]);
    } else {
        const float* c = cyl + 5 * (b - n_sph);
        p = prep_cylinder<double>(t, c[0], c[1], c[2], c[3], c[4]);
    }
    if (body_params_bad(sph, n_sph, cyl, b)) p.ok = 0;
    return p;
}

__device__ __forceinline__ bool finite3(d3 P) { return isfinite(P.x) && isfinite(P.y) && isfinite(P.z); }

// Receiver-side quantities of one body, shared by all of its paths.
//   sphere:   R at polar angle theta_R about e_T in the T-C-R plane, e_perp the
//             in-plane unit normal to e_T towards R; cos/sin of the two
//             detachment polar angles th2_+ = theta_R - gR, th2_- = 2pi - theta_R - gR.
//   cylinder: everything in projection; u2_+ / u2_- the unit directions of the
//             detachment points (R's tangent points) from the axis.
// phi_p is the arc of side + (phi_m = arc_sum - phi_p) with ell = 0.
template <typename G> struct RxGeoT {
    G dR, sD0;            // distance to centre / axis, tangent length
    G phi_p, phi_m;       // arcs of the two sides
    G wn;                 // sphere: distance of R from the source axis
    G along;              // sphere: component of R - C along e_T
    G c2p, s2p, c2m, s2m; // sphere: cos/sin of th2_+/-; cylinder: u2_+/- (x, y)
    V3<G> eperp;          // sphere only
    int ok;               // R outside the body's sphere / circle
};
using RxGeo = RxGeoT<double>;

template <typename G>
__device__ __forceinline__ RxGeoT<G> rx_geo_sphere(const BodyPrepT<G>& b, V3<G> R) {
    RxGeoT<G> g;
    G a = b.a;
    const G idT = grcp(b.dT);
    G cgT = a * idT, sgT = b.sI0 * idT;
    V3<G> C = v3(b.c);
    V3<G> eT = v3(b.eT);
    V3<G> v = R - C;
    G d2 = dot(v, v);
    G along = dot(v, eT);
    g.along = along;
    V3<G> w = v - along * eT;
    g.wn = gnorm(w);
    // on the axis the plane of T, C and R is undefined and w is rounding
    // noise (below a relative 1e-12): any perpendicular serves
    if (g.wn > G(1e-12) * gsqrt(d2)) {
        g.eperp = grcp(g.wn) * w;
    } else {
        d3 ap = any_perp(val3(eT));
        g.eperp = V3<G>{ap.x, ap.y, ap.z};
    }
    g.dR = gsqrt(d2);
    g.ok = g.dR > a;
    g.sD0 = g.ok ? gsqrt((g.dR - a) * (g.dR + a)) : G(0.0);
    G id2 = grcp(d2);
    // th2_+ = theta_R - gR ; th2_- = 2 pi - theta_R - gR
    g.c2p = (along * a + g.wn * g.sD0) * id2;
    g.s2p = (g.wn * a - along * g.sD0) * id2;
    g.c2m = (along * a - g.wn * g.sD0) * id2;
    g.s2m = -(g.wn * a + along * g.sD0) * id2;
    // phi_+ = th2_+ - gT in (-pi, pi)
    G cp = g.c2p * cgT + g.s2p * sgT;
    G sp = g.s2p * cgT - g.c2p * sgT;
    g.phi_p = gatan2(sp, cp);
    G gR = gatan2(g.sD0, a);
    g.phi_m = (kTwoPi - 2.0 * b.gT - 2.0 * gR) - g.phi_p;
    return g;
}

template <typename G>
__device__ __forceinline__ RxGeoT<G> rx_geo_cylinder(const BodyPrepT<G>& b, V3<G> R) {
    RxGeoT<G> g;
    G a = b.a;
    const G idT = grcp(b.dT);
    G cgT = a * idT, sgT = b.sI0 * idT;
    G x = R.x - b.c[0], y = R.y - b.c[1];
    G r2 = x * x + y * y;
    g.dR = gsqrt(r2);
    g.ok = g.dR > a;
    g.sD0 = g.ok ? gsqrt((g.dR - a) * (g.dR + a)) : G(0.0);
    g.wn = G(0.0);
    g.along = G(0.0);
    g.eperp = V3<G>{G(0.0), G(0.0), G(0.0)};
    G ir = grcp(r2);
    // R's tangent points: u_R rotated by -gR (side +) and +gR (side -)
    G cg = a, sg = g.sD0;     // times 1/dR each, folded into ir
    g.c2p = (x * cg + y * sg) * ir;
    g.s2p = (y * cg - x * sg) * ir;
    g.c2m = (x * cg - y * sg) * ir;
    g.s2m = (y * cg + x * sg) * ir;
    // T's tangent point of side +: u_T rotated by +gT
    G u1x = b.eT[0] * cgT - b.eT[1] * sgT, u1y = b.eT[1] * cgT + b.eT[0] * sgT;
    G p = gatan2(u1x * g.s2p - u1y * g.c2p, u1x * g.c2p + u1y * g.s2p);
    G gR = gatan2(g.sD0, a);
    G gsum = b.gT + gR;
    g.phi_p = p >= -gsum ? p : p + kTwoPi;
    g.phi_m = (kTwoPi - 2.0 * gsum) - g.phi_p;
    return g;
}

// Body kinds a kernel handles: both (dispatch on b.kind) or cylinders only.
enum class Kinds { Any, Cylinders };

template <typename G, Kinds K = Kinds::Any>
__device__ __forceinline__ RxGeoT<G> rx_geo(const BodyPrepT<G>& b, V3<G> R) {
    if (K == Kinds::Cylinders || b.kind == 1) return rx_geo_cylinder<G>(b, R);
    return rx_geo_sphere<G>(b, R);
}

// ---------------------------------------------------------------------------
// creeping paths
// ---------------------------------------------------------------------------

// Sphere, side sgn = +1 (towards R) or -1 (far side), ell extra turns.
// Geodesic: great circle in the T-C-R plane; exists when phi >= 0.
// Spreading modulus sqrt(a sin gT / (s^d |rho_perp|)) with |rho_perp| = wn,
// the distance of R from the source axis; one +pi/2 per caustic:
// floor(theta2/pi) surface poles plus one axis crossing when sgn differs from
// the sign of sin(theta2).
template <typename R, typename G>
__device__ __forceinline__ bool sphere_creep(const BodyPrepT<G>& b, const RxGeoT<G>& g, V3<G> Rp, V3<G> T,
                                             const LaunchParams& L, int sgn, int ell, bool* caustic,
                                             PathEvalT<R, G>* pe, PathPts* pts) {
    G phi = (sgn > 0 ? g.phi_p : g.phi_m) + kTwoPi * ell;
    *caustic = false;
    if (!(b.ok && g.ok) || phi < 0.0) return false;
    if (g.wn < L.caustic_guard) { *caustic = true; return false; }
    G a = b.a;
    const G idT = grcp(b.dT);
    G cg = a * idT, sg = b.sI0 * idT;
    G c2 = sgn > 0 ? g.c2p : g.c2m, s2 = sgn > 0 ? g.s2p : g.s2m;
    V3<G> eT = v3(b.eT);
    V3<G> ep = (double)sgn * g.eperp;
    if (pts) {
        V3<G> C = v3(b.c);
        pts->P0 = val3(T);
        pts->P1 = val3(C + a * (cg * eT + sg * ep));
        pts->P2 = val3(C + a * (c2 * eT + s2 * ep));
        pts->P3 = val3(Rp);
    }
    if (pe) {
        G th2 = b.gT + phi;
        int npi = (int)gfloor(th2 * (1.0 / kPi));
        bool s2pos = (npi & 1) == 0;
        int Nc = npi + ((sgn > 0) != s2pos ? 1 : 0);
        G sI = b.sI0, sD = g.sD0;
        pe->s_tot = sI + a * phi + sD;
        pe->nc = Nc;
        // frames in precision R: n1 = cg eT + sg ep, t1 = -sg eT + cg ep,
        // b = t1 x n1 = -(eT x ep), n2 = c2 eT + s2 ep
        R eTx = (R)eT.x, eTy = (R)eT.y, eTz = (R)eT.z;
        R epx = (R)ep.x, epy = (R)ep.y, epz = (R)ep.z;
        R bx = -(eTy * epz - eTz * epy), by = -(eTz * epx - eTx * epz), bz = -(eTx * epy - eTy * epx);
        R cgR = (R)cg, sgR = (R)sg, c2R = (R)c2, s2R = (R)s2;
        R n1x = cgR * eTx + sgR * epx, n1y = cgR * eTy + sgR * epy, n1z = cgR * eTz + sgR * epz;
        R px = (R)L.p[0], py = (R)L.p[1], pz = (R)L.p[2];
        R sIR = (R)sI, sDR = (R)sD, aR = (R)a;
        R Ld = sIR * sDR * RT<R>::rcp(sIR + sDR);
        R mhat = RT<R>::cbrt_((R)0.5 * aR);
        R Smod = RT<R>::sqrt_(aR * sgR * RT<R>::rcp(sDR * (R)g.wn));
        R A = (R)L.amp * Smod * RT<R>::rcp(sIR) * ((R)-1.4142135623730951 * mhat);
        set_fock_consts<R, G>(pe, mhat, (R)phi, Ld);
        R as = A * (px * bx + py * by + pz * bz);
        R ah = A * (px * n1x + py * n1y + pz * n1z);
        pe->vs[0] = as * bx; pe->vs[1] = as * by; pe->vs[2] = as * bz;
        pe->vh[0] = ah * (c2R * eTx + s2R * epx);
        pe->vh[1] = ah * (c2R * eTy + s2R * epy);
        pe->vh[2] = ah * (c2R * eTz + s2R * epz);
        pe->refl = 0;
    }
    return true;
}

// Vertical cylinder: helix that is straight on the unrolled surface.
// L2 = d_T + a phi + d_R, cos(delta) = L2 / sqrt(L2^2 + dz^2), rho_g = a/cos^2,
// xi / m = t / rho_g = phi cos(delta); spreading sqrt(s^i / (s^d (s^i + t + s^d))).
// Valid only if both attachment heights lie on the lateral surface.
template <typename R, typename G>
__device__ __forceinline__ bool cyl_creep(const BodyPrepT<G>& b, const RxGeoT<G>& g, V3<G> Rp, V3<G> T,
                                          const LaunchParams& L, int sgn, int ell, PathEvalT<R, G>* pe,
                                          PathPts* pts) {
    if (!(b.ok && g.ok)) return false;
    G phi = (sgn > 0 ? g.phi_p : g.phi_m) + kTwoPi * ell;
    if (phi < 0.0) return false;
    G a = b.a;
    G dT = b.sI0, dR = g.sD0;
    G L2 = dT + a * phi + dR;
    G dz = Rp.z - T.z;
    const G iL2 = grcp(L2);
    G zQ1 = T.z + dz * dT * iL2;
    G zQ2 = T.z + dz * (dT + a * phi) * iL2;
    if (zQ1 < b.z0 || zQ1 > b.z0 + b.h || zQ2 < b.z0 || zQ2 > b.z0 + b.h) return false;
    const G idT = grcp(b.dT);
    G cgT = a * idT, sgT = b.sI0 * idT;
    // attachment direction: u_T rotated by sgn*gT; detachment: u2 of this side
    G c1 = b.eT[0] * cgT - (double)sgn * b.eT[1] * sgT, s1 = b.eT[1] * cgT + (double)sgn * b.eT[0] * sgT;
    G c2 = sgn > 0 ? g.c2p : g.c2m, s2 = sgn > 0 ? g.s2p : g.s2m;
    if (pts) {
        pts->P0 = val3(T);
        pts->P1 = mk(val(b.c[0] + a * c1), val(b.c[1] + a * s1), val(zQ1));
        pts->P2 = mk(val(b.c[0] + a * c2), val(b.c[1] + a * s2), val(zQ2));
        pts->P3 = val3(Rp);
    }
    if (pe) {
        G Stot = gsqrt(L2 * L2 + dz * dz);
        pe->s_tot = Stot;
        pe->nc = 0;
        const G iS = grcp(Stot);
        R cosd = (R)(L2 * iS), sind = (R)(dz * iS);
        R idc = RT<R>::rcp(cosd);
        R sI = (R)dT * idc, sD = (R)dR * idc;
        R c1R = (R)c1, s1R = (R)s1, c2R = (R)c2, s2R = (R)s2;
        R sg = (R)(double)sgn;
        // t_i = cosd * sgn (-s_i, c_i, 0) + sind z;  b_i = t_i x n_i, n_i = (c_i, s_i, 0)
        R b1x = -sind * s1R, b1y = sind * c1R, b1z = -cosd * sg;
        R b2x = -sind * s2R, b2y = sind * c2R, b2z = b1z;
        R rho_g = (R)a * idc * idc;
        R mhat = RT<R>::cbrt_((R)0.5 * rho_g);
        R Ld = sI * sD * RT<R>::rcp(sI + sD);
        R Smod = RT<R>::sqrt_(sI * RT<R>::rcp(sD * (R)Stot));
        R px = (R)L.p[0], py = (R)L.p[1], pz = (R)L.p[2];
        R A = (R)L.amp * Smod * RT<R>::rcp(sI) * ((R)-1.4142135623730951 * mhat);
        set_fock_consts<R, G>(pe, mhat, (R)phi * cosd, Ld);
        R as = A * (px * b1x + py * b1y + pz * b1z);
        R ah = A * (px * c1R + py * s1R);
        pe->vs[0] = as * b2x; pe->vs[1] = as * b2y; pe->vs[2] = as * b2z;
        pe->vh[0] = ah * c2R; pe->vh[1] = ah * s2R; pe->vh[2] = (R)0;
        pe->refl = 0;
    }
    return true;
}

// ---------------------------------------------------------------------------
// reflection
// ---------------------------------------------------------------------------

// Stationarity condition of Alhazen's problem on a circle of radius a
// centred at the origin: with Q = a (cos th, sin th),
// g(th) = d/dth (|Q - P1| + |Q - P2|) / a = (Q - P1).t/|Q - P1| + (Q - P2).t/|Q - P2|,
// t the unit tangent; *dg = g'(th).
template <typename G>
__device__ __forceinline__ G alhazen_fun(G a, G p1x, G p1y, G p2x, G p2y, G th, G* dg) {
    G s, c;
    gsincos(th, &s, &c);
    G qx = a * c, qy = a * s;
    G d1x = qx - p1x, d1y = qy - p1y, d2x = qx - p2x, d2y = qy - p2y;
    G i1 = grsqrt(d1x * d1x + d1y * d1y), i2 = grsqrt(d2x * d2x + d2y * d2y);   // 1/|Q - P|
    G t1 = (-d1x * s + d1y * c) * i1, t2 = (-d2x * s + d2y * c) * i2;   // unit (Q-P).t
    G n1 = d1x * c + d1y * s, n2 = d2x * c + d2y * s;                  // (Q-P).n
    *dg = ((a - n1) - a * t1 * t1) * i1 + ((a - n2) - a * t2 * t2) * i2;
    return t1 + t2;
}

// The same function in FP32 (hardware sin/cos of revolutions, reciprocal
// square roots): good to about 1e-6 in th, enough to start the FP64 polish
// within its quadratic range.
__device__ __forceinline__ float alhazen_fun_f32(float a, float p1x, float p1y, float p2x, float p2y, float th,
                                                 float* dg) {
    float r = th * 0.159154943091895336f;
    r -= rintf(r);
    float s, c;
    sincos_rev(r, &s, &c);
    const float qx = a * c, qy = a * s;
    const float d1x = qx - p1x, d1y = qy - p1y, d2x = qx - p2x, d2y = qy - p2y;
    const float i1 = __builtin_amdgcn_rsqf(d1x * d1x + d1y * d1y), i2 = __builtin_amdgcn_rsqf(d2x * d2x + d2y * d2y);
    const float t1 = (-d1x * s + d1y * c) * i1, t2 = (-d2x * s + d2y * c) * i2;
    const float n1 = d1x * c + d1y * s, n2 = d2x * c + d2y * s;
    *dg = ((a - n1) - a * t1 * t1) * i1 + ((a - n2) - a * t2 * t2) * i2;
    return t1 + t2;
}

// Root of g between the tangent points lo and hi (either order; g has
// opposite signs there).  Safeguarded Newton (a bisection step whenever
// Newton leaves the bracket) in FP32 to about 1e-6, then the same in FP64
// from there.  The FP64 iteration stops after a Newton step below
// 1e-11 (1 + |th|): with quadratic convergence the accepted iterate is then
// exact to far below FP64 rounding.  Typically 4-5 FP32 and 2-3 FP64
// evaluations.  With FULL = false (paths whose constants are FP32) one FP64
// Newton step from the FP32 root is accepted when it is below
// 1e-5 (1 + |th|): the root is then within about 1e-9 rad (far inside the FP32
// constants, and the path length is stationary in th); otherwise the full
// iteration runs.
template <bool FULL = true>
__device__ __forceinline__ double alhazen(double a, double p1x, double p1y, double p2x, double p2y,
                                          double lo, double hi) {
    const float fa = (float)a, f1x = (float)p1x, f1y = (float)p1y, f2x = (float)p2x, f2y = (float)p2y;
    float flo = (float)lo, fhi = (float)hi, fdg;
    const float glo32 = alhazen_fun_f32(fa, f1x, f1y, f2x, f2y, flo, &fdg);
    float fg_lo = glo32;
    float fth = 0.5f * (flo + fhi);
    for (int it = 0; it < 40; ++it) {
        const float g = alhazen_fun_f32(fa, f1x, f1y, f2x, f2y, fth, &fdg);
        if (g == 0.0f) break;
        if ((g < 0.0f) == (fg_lo < 0.0f)) { flo = fth; fg_lo = g; } else { fhi = fth; }
        float nt = fth - g * __builtin_amdgcn_rcpf(fdg);
        const float tol = 2e-6f * (1.0f + fabsf(fth));
        if (fabsf(nt - fth) <= tol) { fth = nt; break; }
        if (!(nt > fminf(flo, fhi) && nt < fmaxf(flo, fhi))) nt = 0.5f * (flo + fhi);
        fth = nt;
        if (fabsf(fhi - flo) <= tol) break;
    }
    double dg;
    if (!FULL) {
        const double th0 = (double)fth;
        if (th0 > fmin(lo, hi) && th0 < fmax(lo, hi)) {
            const double g = alhazen_fun<double>(a, p1x, p1y, p2x, p2y, th0, &dg);
            const double nt = th0 - g / dg;
            if (fabs(nt - th0) <= 1e-5 * (1.0 + fabs(th0)) && nt > fmin(lo, hi) && nt < fmax(lo, hi)) return nt;
        }
    }
    // sign of g at lo: from the FP32 value unless that is too small to trust
    bool lo_neg = glo32 < 0.0f;
    if (fabsf(glo32) < 1e-4f) lo_neg = alhazen_fun<double>(a, p1x, p1y, p2x, p2y, lo, &dg) < 0.0;
    double th = (double)fth;
    if (!(th > fmin(lo, hi) && th < fmax(lo, hi))) th = 0.5 * (lo + hi);
    for (int it = 0; it < 60; ++it) {
        const double g = alhazen_fun<double>(a, p1x, p1y, p2x, p2y, th, &dg);
        if (g == 0.0) break;
        if ((g < 0) == lo_neg) lo = th; else hi = th;
        double nt = th - g * grcp(dg);
        if (fabs(nt - th) <= 1e-11 * (1.0 + fabs(th))) { th = nt; break; }
        if (!(nt > fmin(lo, hi) && nt < fmax(lo, hi))) nt = 0.5 * (lo + hi);
        th = nt;
        if (fabs(hi - lo) <= 1e-15 * (1.0 + fabs(th))) break;
    }
    return th;
}

// Whether a finite vertical cylinder can carry any path to the receiver at
// all, from distances alone (no angles): a creeping path needs both its
// attachment heights on the lateral surface, z_Q1 = z_T + dz d_T / L2 and
// z_Q2 = z_T + dz (1 - d_R / L2), with L2 = d_T + a phi + d_R and
// 0 <= phi < 2 pi (l_enc + 1) (d_T, d_R the tangent lengths); a reflection
// needs its point's height (bounded as in refl_angle) there.  False only
// when every such height range misses the surface, so the classification
// (two atan2 per pair) can be skipped; a necessary condition, never a
// sufficient one.
__device__ __forceinline__ bool cyl_paths_possible(const BodyPrep& b, d3 Rp, d3 T, const LaunchParams& L) {
    if (!b.ok) return false;
    const double x = Rp.x - b.c[0], y = Rp.y - b.c[1];
    const double a = b.a, dR = sqrt(x * x + y * y);
    if (!(dR > a)) return false;
    const double sD = sqrt((dR - a) * (dR + a));
    const double dz = Rp.z - T.z;
    const double slack = 1e-9 * (1.0 + fabs(T.z) + fabs(Rp.z));
    const double zlo = b.z0 - slack, zhi = b.z0 + b.h + slack;
    // z = z_T + dz f over f between fa and fb meets [zlo, zhi]
    auto meets = [&](double fa, double fb) {
        const double za = T.z + dz * fa, zb = T.z + dz * fb;
        return fmax(za, zb) >= zlo && fmin(za, zb) <= zhi;
    };
    // reciprocals within a few ulp: far below the slack
    const double l0 = b.sI0 + sD, l1 = l0 + kTwoPi * (L.l_enc + 1) * a;
    const double il0 = grcp(l0), il1 = grcp(l1);
    if (meets(b.sI0 * il1, b.sI0 * il0) && meets(1.0 - sD * il0, 1.0 - sD * il1)) return true;
    if (L.lit_branch) {
        const double fa = (b.dT - a) * grcp((b.dT - a) + sD), fb = b.sI0 * grcp(b.sI0 + (dR - a));
        if (meets(fa, fb)) return true;
    }
    return false;
}

// cyl_paths_possible for every receiver of a box at once: false only when
// no receiver with lo <= R <= hi (componentwise) passes it.  The distances
// to the axis over the box bound the tangent lengths, and each height test
// becomes the range of z_T + dz f over the box of (dz, f) that the
// receivers' values fill; the slack is a thousand times the per-receiver one.
__device__ __forceinline__ bool cyl_box_possible(const BodyPrep& b, const float* lo, const float* hi, d3 T,
                                                 const LaunchParams& L) {
    if (!b.ok) return false;
    const double a = b.a;
    const double ex = fmax(fmax((double)lo[0] - b.c[0], b.c[0] - (double)hi[0]), 0.0);
    const double ey = fmax(fmax((double)lo[1] - b.c[1], b.c[1] - (double)hi[1]), 0.0);
    const double fx = fmax(fabs((double)lo[0] - b.c[0]), fabs((double)hi[0] - b.c[0]));
    const double fy = fmax(fabs((double)lo[1] - b.c[1]), fabs((double)hi[1] - b.c[1]));
    const double dmax = sqrt(fx * fx + fy * fy);
    if (!(dmax > a)) return false;
    const double d0 = fmax(sqrt(ex * ex + ey * ey), a);
    const double s0 = sqrt(fmax((d0 - a) * (d0 + a), 0.0)), s1 = sqrt((dmax - a) * (dmax + a));
    const double dz0 = (double)lo[2] - T.z, dz1 = (double)hi[2] - T.z;
    const double slack = 1e-6 * (1.0 + fabs(T.z) + fmax(fabs((double)lo[2]), fabs((double)hi[2])));
    const double zlo = b.z0 - slack, zhi = b.z0 + b.h + slack;
    auto meets = [&](double f0, double f1) {
        const double p0 = dz0 * f0, p1 = dz0 * f1, p2 = dz1 * f0, p3 = dz1 * f1;
        return T.z + fmax(fmax(p0, p1), fmax(p2, p3)) >= zlo && T.z + fmin(fmin(p0, p1), fmin(p2, p3)) <= zhi;
    };
    const double sI = b.sI0, c = kTwoPi * (L.l_enc + 1) * a;
    if (meets(sI / (sI + s1 + c), sI / (sI + s0)) && meets(sI / (sI + s1), 1.0 - s0 / (sI + s0 + c))) return true;
    if (L.lit_branch) {
        const double da = b.dT - a;
        const double fa0 = da / (da + s1), fa1 = da / (da + s0);
        const double fb0 = sI / (sI + (dmax - a)), fb1 = sI / (sI + (d0 - a));
        if (meets(fmin(fa0, fb0), fmax(fa1, fb1))) return true;
    }
    return false;
}

// Reflection point for a lit receiver: the angle parameter (sphere: polar
// angle in the T-C-R plane; cylinder: azimuth), false if the receiver is not
// lit by this body or the point is off the lateral surface.
template <Kinds K = Kinds::Any, bool FULL = true>
__device__ __forceinline__ bool refl_angle(const BodyPrep& b, const RxGeo& g, d3 Rp, d3 T, double* th_out) {
    if (!(b.ok && g.ok)) return false;
    double a = b.a;
    if (K == Kinds::Any && b.kind == 0) {
        if (!(g.phi_p < 0)) return false;
        // T at (dT, 0), R at (along, wn) in the plane basis; the arc seen
        // from both runs from R's tangent point (thR - gR = phi_+ + gT) to T's (gT)
        *th_out = alhazen<FULL>(a, b.dT, 0.0, g.along, g.wn, g.phi_p + b.gT, b.gT);
        return true;
    }
    double lo, hi;
    if (g.phi_p < 0) {
        lo = b.aT + g.phi_p + b.gT;      // = aT + dphi_+ - gR
        hi = b.aT + b.gT;
    } else if (g.phi_m < 0) {
        lo = b.aT - b.gT;
        hi = b.aT - g.phi_m - b.gT;      // = aT - dphi_- + gR
    } else {
        return false;
    }
    // Height of the reflection point before solving: on the arc seen from
    // both ends, the horizontal distances obey rho_T - a <= l_T <= s_T and
    // rho_R - a <= l_R <= s_R (s the tangent lengths), so
    // z_Q = z_T + (z_R - z_T) l_T / (l_T + l_R) lies between the values at
    // the extreme ratios; no solve when that range misses the lateral surface.
    {
        const double fa = (b.dT - a) * grcp((b.dT - a) + g.sD0), fb = b.sI0 * grcp(b.sI0 + (g.dR - a));
        const double dz = Rp.z - T.z;
        const double za = T.z + dz * fa, zb = T.z + dz * fb;
        const double slack = 1e-9 * (1.0 + fabs(T.z) + fabs(Rp.z));
        if (fmax(za, zb) < b.z0 - slack || fmin(za, zb) > b.z0 + b.h + slack) return false;
    }
    double tx = T.x - b.c[0], ty = T.y - b.c[1];
    double rx = Rp.x - b.c[0], ry = Rp.y - b.c[1];
    double al = alhazen<FULL>(a, tx, ty, rx, ry, lo, hi);
    double s, c;
    gsincos(al, &s, &c);
    double qx = a * c, qy = a * s;
    double lt = sqrt((qx - tx) * (qx - tx) + (qy - ty) * (qy - ty));
    double lr = sqrt((qx - rx) * (qx - rx) + (qy - ry) * (qy - ry));
    double zQ = T.z + (Rp.z - T.z) * lt * grcp(lt + lr);
    if (zQ < b.z0 || zQ > b.z0 + b.h) return false;
    *th_out = al;
    return true;
}

// The reflection angle as a function of the geometry: one Newton step from
// the converged FP64 root th, taken in G.  For a dual G the step carries
// d th = -(dg/dp) / g'(th) (implicit differentiation of g(th, p) = 0).
template <typename G>
__device__ __forceinline__ G refl_angle_g(const BodyPrepT<G>& b, const RxGeoT<G>& g, V3<G> Rp, V3<G> T, double th) {
    G dg;
    G r;
    if (b.kind == 0)
        r = alhazen_fun<G>(b.a, b.dT, G(0.0), g.along, g.wn, G(th), &dg);
    else
        r = alhazen_fun<G>(b.a, T.x - b.c[0], T.y - b.c[1], Rp.x - b.c[0], Rp.y - b.c[1], G(th), &dg);
    return G(th) - r / G(val(dg));
}

// Reflection point and its normal from the angle.
template <typename G, Kinds K = Kinds::Any>
__device__ __forceinline__ void refl_point(const BodyPrepT<G>& b, const RxGeoT<G>& g, V3<G> Rp, V3<G> T, G th,
                                           V3<G>* Q, V3<G>* n) {
    G s, c;
    gsincos(th, &s, &c);
    V3<G> q, nn;   // written once at the end: keeps both in registers
    if (K == Kinds::Any && b.kind == 0) {
        V3<G> eT = v3(b.eT);
        nn = c * eT + s * g.eperp;
        q = v3(b.c) + b.a * nn;
    } else {
        G a = b.a;
        G tx = T.x - b.c[0], ty = T.y - b.c[1];
        G rx = Rp.x - b.c[0], ry = Rp.y - b.c[1];
        G qx = a * c, qy = a * s;
        G lt = gsqrt((qx - tx) * (qx - tx) + (qy - ty) * (qy - ty));
        G lr = gsqrt((qx - rx) * (qx - rx) + (qy - ry) * (qy - ry));
        G zQ = T.z + (Rp.z - T.z) * lt * grcp(lt + lr);
        q = V3<G>{b.c[0] + qx, b.c[1] + qy, zQ};
        nn = V3<G>{c, s, G(0.0)};
    }
    *Q = q;
    *n = nn;
}

// Reflected-field constants.  Caustic distances written as
// 1/rho_1 = 1/s^i + f1/cos(th_i), 1/rho_2 = 1/s^i + f2 cos(th_i)
// (sphere: f1 = f2 = 2/a, rho_g = a; cylinder: f1 = 2 cos^2(beta)/a, f2 = 0,
// rho_g = a / cos^2(delta_R)).
template <typename R, typename G>
__device__ __forceinline__ void refl_eval(const BodyPrepT<G>& b, V3<G> Q, V3<G> n, V3<G> Rp, V3<G> T,
                                          const LaunchParams& L, PathEvalT<R, G>* pe) {
    V3<G> vi = Q - T, vr = Rp - Q;
    G sI = gnorm(vi), sR = gnorm(vr);
    pe->s_tot = sI + sR;
    pe->nc = 0;
    R isI = (R)grcp(sI), isR = (R)grcp(sR);
    R six = (R)vi.x * isI, siy = (R)vi.y * isI, siz = (R)vi.z * isI;
    R srx = (R)vr.x * isR, sry = (R)vr.y * isR, srz = (R)vr.z * isR;
    R nx = (R)n.x, ny = (R)n.y, nz = (R)n.z;
    R ci = -(six * nx + siy * ny + siz * nz);
    ci = ci < (R)0 ? (R)0 : (ci > (R)1 ? (R)1 : ci);
    R a = (R)b.a;
    R rho_g, f1, f2;
    if (b.kind == 0) {
        rho_g = a;
        f1 = (R)2 * RT<R>::rcp(a);
        f2 = f1;
    } else {
        // circumferential unit (-n_y, n_x, 0); trace of the incidence plane
        R sn = six * nx + siy * ny + siz * nz;
        R tgx = six - sn * nx, tgy = siy - sn * ny, tgz = siz - sn * nz;
        R tn2 = tgx * tgx + tgy * tgy + tgz * tgz;
        R tc = -tgx * ny + tgy * nx;
        R cos2d = tn2 > (R)0 ? tc * tc * RT<R>::rcp(tn2) : (R)1;
        cos2d = cos2d < (R)1e-12 ? (R)1e-12 : cos2d;
        rho_g = a * RT<R>::rcp(cos2d);
        f1 = (R)2 * ((R)1 - siz * siz) * RT<R>::rcp(a);
        f2 = (R)0;
    }
    R sIR = (R)sI, sRR = (R)sR;
    R r1c = RT<R>::rcp(ci * isI + f1);
    R rho1 = r1c * ci;
    R rho2 = RT<R>::rcp(isI + f2 * ci);
    // e_perp = s_i x n / |.|, e_par^i = e_perp x s_i, e_par^r = e_perp x s_r
    R cx = siy * nz - siz * ny, cy = siz * nx - six * nz, cz = six * ny - siy * nx;
    R cn = RT<R>::sqrt_(cx * cx + cy * cy + cz * cz);
    if (cn > (R)1e-6) {
        R ic = RT<R>::rcp(cn);
        cx *= ic; cy *= ic; cz *= ic;
    } else {
        d3 ap = any_perp(val3(n));
        cx = (R)ap.x; cy = (R)ap.y; cz = (R)ap.z;
    }
    R pix = cy * siz - cz * siy, piy = cz * six - cx * siz, piz = cx * siy - cy * six;
    R prx = cy * srz - cz * sry, pry = cz * srx - cx * srz, prz = cx * sry - cy * srx;
    R mhat = RT<R>::cbrt_((R)0.5 * rho_g);
    R Lr = sIR * sRR * RT<R>::rcp(sIR + sRR);
    R P0 = (R)2 * RT<R>::sqrt_(r1c * RT<R>::rcp((R)2 * mhat)) *
           RT<R>::sqrt_(rho2 * RT<R>::rcp((rho1 + sRR) * (rho2 + sRR)));
    R px = (R)L.p[0], py = (R)L.p[1], pz = (R)L.p[2];
    R A = (R)L.amp * isI * P0;
    set_fock_consts<R, G>(pe, mhat, (R)-2 * ci, Lr);
    R as = A * (px * cx + py * cy + pz * cz);
    R ah = A * (px * pix + py * piy + pz * piz);
    pe->vs[0] = as * cx; pe->vs[1] = as * cy; pe->vs[2] = as * cz;
    pe->vh[0] = ah * prx; pe->vh[1] = ah * pry; pe->vh[2] = ah * prz;
    pe->refl = 1;
}

}  // namespace utd

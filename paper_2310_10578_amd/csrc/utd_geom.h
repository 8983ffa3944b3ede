// Ray geometry of the smooth-surface UTD paths on spheres and vertical
// cylinders (device code).  Lengths, angles and the reflection-point root
// solve are carried in FP64; the frequency-independent path constants handed
// to the frequency loop are rounded to the field precision R.
//
// Creeping path (Eq. (4), Sec. III-B): tangent from the source T to the
// attachment point Q1, surface geodesic Q1 -> Q2 of length t, tangent from
// the detachment point Q2 to the receiver R.
// Reflection (Eq. (3)): the specular point Q_R on the arc seen from both T
// and R.
#pragma once

#include "utd_device.h"

namespace utd {

// Everything the frequency loop needs about one path.  The per-frequency
// coefficient is  K_p(xi, X) with xi = mhat k^{1/3} phi_e, X = k Lh phi_e^2,
// q = k^{1/6} qhat, and the contribution is
//   e^{-j 2pi rev} k^{-1/6} (a_s K_s v_s + a_h K_h v_h),  rev = k s_tot / 2pi + rev0.
template <typename R> struct PathEval {
    double s_tot;     // total path length s^i + t + s^d (or s^i + s^r)
    double rev0;      // extra phase in revolutions (caustics: -N_c/4)
    R phi_e, mhat, Lh, qhat;
    R a_s, a_h;       // incident projections x spreading x prefactor
    R vs[3], vh[3];   // output polarisation vectors at R
    int refl;
};

// Points of a path (for the visibility tests).
struct PathPts {
    d3 P0, P1;        // first leg  T -> Q1 (or Q_R)
    d3 P2, P3;        // second leg Q2 (or Q_R) -> R
};

__device__ __forceinline__ BodyPrep body_prep(const double T[3], const float* sph, int n_sph,
                                              const float* cyl, int b) {
    BodyPrep p;
    p.pad[0] = p.pad[1] = 0;
    d3 t = mk(T[0], T[1], T[2]);
    if (b < n_sph) {
        const float* s = sph + 4 * b;
        p.kind = 0;
        p.c[0] = s[0]; p.c[1] = s[1]; p.c[2] = s[2];
        p.a = s[3];
        p.z0 = 0; p.h = 0;
        d3 v = t - mk(p.c[0], p.c[1], p.c[2]);
        p.dT = norm(v);
        d3 e = (1.0 / p.dT) * v;
        p.eT[0] = e.x; p.eT[1] = e.y; p.eT[2] = e.z;
        p.ok = p.dT > p.a;
        p.sI0 = p.ok ? sqrt((p.dT - p.a) * (p.dT + p.a)) : 0.0;
        p.gT = atan2(p.sI0, p.a);
        p.aT = 0;
    } else {
        const float* c = cyl + 5 * (b - n_sph);
        p.kind = 1;
        p.c[0] = c[0]; p.c[1] = c[1]; p.c[2] = 0;
        p.z0 = c[2]; p.h = c[3]; p.a = c[4];
        double tx = T[0] - p.c[0], ty = T[1] - p.c[1];
        p.dT = sqrt(tx * tx + ty * ty);
        p.eT[0] = tx / p.dT; p.eT[1] = ty / p.dT; p.eT[2] = 0;
        p.ok = p.dT > p.a;
        p.sI0 = p.ok ? sqrt((p.dT - p.a) * (p.dT + p.a)) : 0.0;
        p.gT = atan2(p.sI0, p.a);
        p.aT = atan2(ty, tx);
    }
    return p;
}

__device__ __forceinline__ bool inside_body(const BodyPrep& b, d3 P) {
    if (b.kind == 0) {
        d3 v = P - mk(b.c[0], b.c[1], b.c[2]);
        return dot(v, v) <= b.a * b.a;
    }
    double x = P.x - b.c[0], y = P.y - b.c[1];
    return x * x + y * y <= b.a * b.a && P.z >= b.z0 && P.z <= b.z0 + b.h;
}

// Receiver-side quantities of one body, shared by its paths.
struct RxGeo {
    // sphere: along = e_T.(R-C), wn = |perp|, e_perp; cylinder: xy offsets
    double dR, sD0, gR;      // distance (to centre / axis), tangent length, half-angle
    double thR;              // sphere: polar angle of R about e_T
    double dphi_plus;        // cylinder: CCW angle from T to R about the axis
    double along, wn;
    d3 eperp;
    int ok;                  // receiver outside the body's sphere / circle
};

__device__ __forceinline__ RxGeo rx_geo(const BodyPrep& b, d3 R) {
    RxGeo g;
    if (b.kind == 0) {
        d3 C = mk(b.c[0], b.c[1], b.c[2]);
        d3 eT = mk(b.eT[0], b.eT[1], b.eT[2]);
        d3 v = R - C;
        g.dR = norm(v);
        g.along = dot(v, eT);
        d3 w = v - g.along * eT;
        g.wn = norm(w);
        g.eperp = g.wn > 1e-300 ? (1.0 / g.wn) * w : any_perp(eT);
        g.thR = atan2(g.wn, g.along);
        g.dphi_plus = 0;
    } else {
        double x = R.x - b.c[0], y = R.y - b.c[1];
        g.dR = sqrt(x * x + y * y);
        double aR = atan2(y, x);
        double d = aR - b.aT;
        d = d - kTwoPi * floor(d * kInvTwoPi);
        if (d >= kTwoPi) d -= kTwoPi;
        g.dphi_plus = d;
        g.thR = 0; g.along = 0; g.wn = 0;
        g.eperp = mk(0, 0, 0);
    }
    g.ok = g.dR > b.a;
    g.sD0 = g.ok ? sqrt((g.dR - b.a) * (g.dR + b.a)) : 0.0;
    g.gR = atan2(g.sD0, b.a);
    return g;
}

// ---------------------------------------------------------------------------
// creeping paths
// ---------------------------------------------------------------------------

// Sphere, side sgn = +1 (towards R) or -1 (far side), ell extra turns.
// Geodesic: great circle in the T-C-R plane, arc phi = theta_R - gT - gR
// (side +) or 2 pi - theta_R - gT - gR (side -), plus 2 pi ell; exists when
// phi >= 0.  Spreading modulus sqrt(a sin gT / (s^d |rho_perp|)) with
// |rho_perp| = |R - axis| = wn; one +pi/2 per caustic: floor(theta2/pi)
// surface poles plus one axis crossing when sgn differs from sign(sin theta2).
template <typename R>
__device__ __forceinline__ bool sphere_creep(const BodyPrep& b, const RxGeo& g, d3 Rp, const LaunchParams& L,
                                             int sgn, int ell, bool* caustic, PathEval<R>* pe, PathPts* pts) {
    double phi = (sgn > 0 ? g.thR : kTwoPi - g.thR) - b.gT - g.gR + kTwoPi * ell;
    *caustic = false;
    if (!(b.ok && g.ok) || phi < 0) return false;
    if (g.wn < L.caustic_guard) { *caustic = true; return false; }
    double a = b.a;
    d3 C = mk(b.c[0], b.c[1], b.c[2]);
    d3 eT = mk(b.eT[0], b.eT[1], b.eT[2]);
    d3 ep = (double)sgn * g.eperp;
    double cg = a / b.dT, sg = b.sI0 / b.dT;
    double th2 = b.gT + phi;
    double s2, c2;
    sincos(th2, &s2, &c2);
    d3 n1 = cg * eT + sg * ep;
    d3 t1 = (-sg) * eT + cg * ep;
    d3 n2 = c2 * eT + s2 * ep;
    d3 bb = cross(t1, n1);
    if (pts) {
        pts->P0 = mk(L.T[0], L.T[1], L.T[2]);
        pts->P1 = C + a * n1;
        pts->P2 = C + a * n2;
        pts->P3 = Rp;
    }
    if (pe) {
        double np = floor(th2 * (1.0 / kPi));
        int npi = (int)np;
        bool s2pos = (npi & 1) == 0;
        int Nc = npi + ((sgn > 0) != s2pos ? 1 : 0);
        double sI = b.sI0, sD = g.sD0;
        double Smod = sqrt(a * sg / (sD * g.wn));
        double mhat = cbrt(0.5 * a);
        double Ld = sI * sD / (sI + sD);
        d3 p = mk(L.p[0], L.p[1], L.p[2]);
        double A = L.amp * Smod / sI;
        double P0 = -1.4142135623730951 * mhat;
        pe->s_tot = sI + a * phi + sD;
        pe->rev0 = -0.25 * Nc;
        pe->phi_e = (R)phi;
        pe->mhat = (R)mhat;
        pe->Lh = (R)(0.5 * Ld);
        pe->qhat = (R)(sqrt(0.5 * Ld) / mhat);
        pe->a_s = (R)(A * dot(p, bb) * P0);
        pe->a_h = (R)(A * dot(p, n1) * P0);
        pe->vs[0] = (R)bb.x; pe->vs[1] = (R)bb.y; pe->vs[2] = (R)bb.z;
        pe->vh[0] = (R)n2.x; pe->vh[1] = (R)n2.y; pe->vh[2] = (R)n2.z;
        pe->refl = 0;
    }
    return true;
}

// Vertical cylinder: helix that is straight on the unrolled surface.
// L2 = d_T + a phi + d_R, cos(delta) = L2 / sqrt(L2^2 + dz^2), rho_g = a/cos^2,
// xi / m = t / rho_g = phi cos(delta); spreading sqrt(s^i / (s^d (s^i + t + s^d))).
// Valid only if both attachment heights lie on the lateral surface.
template <typename R>
__device__ __forceinline__ bool cyl_creep(const BodyPrep& b, const RxGeo& g, d3 Rp, const LaunchParams& L,
                                          int sgn, int ell, PathEval<R>* pe, PathPts* pts) {
    if (!(b.ok && g.ok)) return false;
    double dphi = sgn > 0 ? g.dphi_plus : kTwoPi - g.dphi_plus;
    double phi = dphi - b.gT - g.gR + kTwoPi * ell;
    if (phi < 0) return false;
    double a = b.a;
    double dT = b.sI0, dR = g.sD0;
    double L2 = dT + a * phi + dR;
    double dz = Rp.z - L.T[2];
    double Stot = sqrt(L2 * L2 + dz * dz);
    double zQ1 = L.T[2] + dz * dT / L2;
    double zQ2 = L.T[2] + dz * (dT + a * phi) / L2;
    if (zQ1 < b.z0 || zQ1 > b.z0 + b.h || zQ2 < b.z0 || zQ2 > b.z0 + b.h) return false;
    double al1 = b.aT + sgn * b.gT;
    double al2 = al1 + sgn * phi;
    double s1, c1, s2, c2;
    sincos(al1, &s1, &c1);
    sincos(al2, &s2, &c2);
    if (pts) {
        pts->P0 = mk(L.T[0], L.T[1], L.T[2]);
        pts->P1 = mk(b.c[0] + a * c1, b.c[1] + a * s1, zQ1);
        pts->P2 = mk(b.c[0] + a * c2, b.c[1] + a * s2, zQ2);
        pts->P3 = Rp;
    }
    if (pe) {
        double cosd = L2 / Stot, sind = dz / Stot;
        double sI = dT / cosd, t = a * phi / cosd, sD = dR / cosd;
        d3 n1 = mk(c1, s1, 0), n2 = mk(c2, s2, 0);
        d3 t1 = mk(-sgn * cosd * s1, sgn * cosd * c1, sind);
        d3 t2 = mk(-sgn * cosd * s2, sgn * cosd * c2, sind);
        d3 b1 = cross(t1, n1), b2 = cross(t2, n2);
        double rho_g = a / (cosd * cosd);
        double mhat = cbrt(0.5 * rho_g);
        double Ld = sI * sD / (sI + sD);
        double Smod = sqrt(sI / (sD * Stot));
        d3 p = mk(L.p[0], L.p[1], L.p[2]);
        double A = L.amp * Smod / sI;
        double P0 = -1.4142135623730951 * mhat;
        pe->s_tot = Stot;
        pe->rev0 = 0.0;
        pe->phi_e = (R)(phi * cosd);
        pe->mhat = (R)mhat;
        pe->Lh = (R)(0.5 * Ld);
        pe->qhat = (R)(sqrt(0.5 * Ld) / mhat);
        pe->a_s = (R)(A * dot(p, b1) * P0);
        pe->a_h = (R)(A * dot(p, n1) * P0);
        pe->vs[0] = (R)b2.x; pe->vs[1] = (R)b2.y; pe->vs[2] = (R)b2.z;
        pe->vh[0] = (R)n2.x; pe->vh[1] = (R)n2.y; pe->vh[2] = (R)n2.z;
        (void)t;
        pe->refl = 0;
    }
    return true;
}

// ---------------------------------------------------------------------------
// reflection
// ---------------------------------------------------------------------------

// Alhazen's problem on a circle of radius a centred at the origin: the point
// Q = a (cos th, sin th), th in [lo, hi], where d/dth (|Q - P1| + |Q - P2|) = 0.
// Safeguarded Newton in FP64 (bisection step whenever Newton leaves the
// bracket); the bracket ends are the tangent points, where the derivative has
// opposite signs.
__device__ __forceinline__ double alhazen(double a, double p1x, double p1y, double p2x, double p2y,
                                          double lo, double hi) {
    auto gfun = [&](double th, double* dg) {
        double s, c;
        sincos(th, &s, &c);
        double qx = a * c, qy = a * s;
        double d1x = qx - p1x, d1y = qy - p1y, d2x = qx - p2x, d2y = qy - p2y;
        double l1 = sqrt(d1x * d1x + d1y * d1y), l2 = sqrt(d2x * d2x + d2y * d2y);
        double t1 = -d1x * s + d1y * c, t2 = -d2x * s + d2y * c;      // (Q-P).t
        double n1 = d1x * c + d1y * s, n2 = d2x * c + d2y * s;        // (Q-P).n
        double g = t1 / l1 + t2 / l2;
        *dg = (a - n1) / l1 - a * t1 * t1 / (l1 * l1 * l1) + (a - n2) / l2 - a * t2 * t2 / (l2 * l2 * l2);
        return g;
    };
    double dg;
    double glo = gfun(lo, &dg);
    double th = 0.5 * (lo + hi);
    for (int it = 0; it < 60; ++it) {
        double g = gfun(th, &dg);
        if ((g < 0) == (glo < 0)) { lo = th; glo = g; } else { hi = th; }
        double nt = th - g / dg;
        if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
        if (fabs(nt - th) <= 1e-15 * (1.0 + fabs(th)) || hi - lo <= 1e-15 * (1.0 + fabs(th))) { th = nt; break; }
        th = nt;
    }
    return th;
}

// Shared reflection bookkeeping; caustic distances written as
// 1/rho_1 = 1/s^i + f1/cos(th_i), 1/rho_2 = 1/s^i + f2 cos(th_i)
// (sphere: f1 = f2 = 2/a; cylinder: f1 = 2 cos^2(beta)/a, f2 = 0).
template <typename R>
__device__ __forceinline__ void refl_common(d3 T, d3 Q, d3 n, d3 Rp, double rho_g, double f1, double f2,
                                            const LaunchParams& L, PathEval<R>* pe) {
    d3 vi = Q - T, vr = Rp - Q;
    double sI = norm(vi), sR = norm(vr);
    d3 si = (1.0 / sI) * vi, sr = (1.0 / sR) * vr;
    double ci = -dot(si, n);
    ci = ci < 0 ? 0 : (ci > 1 ? 1 : ci);
    double r1c = 1.0 / (ci / sI + f1);
    double rho1 = r1c * ci;
    double rho2 = 1.0 / (1.0 / sI + f2 * ci);
    d3 cr = cross(si, n);
    double crn = norm(cr);
    d3 eperp = crn > 1e-12 ? (1.0 / crn) * cr : any_perp(n);
    d3 epi = cross(eperp, si), epr = cross(eperp, sr);
    double mhat = cbrt(0.5 * rho_g);
    double Lr = sI * sR / (sI + sR);
    double P0 = 2.0 * sqrt(r1c / (2.0 * mhat)) * sqrt(rho2 / ((rho1 + sR) * (rho2 + sR)));
    d3 p = mk(L.p[0], L.p[1], L.p[2]);
    double A = L.amp / sI * P0;
    pe->s_tot = sI + sR;
    pe->rev0 = 0.0;
    pe->phi_e = (R)(-2.0 * ci);
    pe->mhat = (R)mhat;
    pe->Lh = (R)(0.5 * Lr);
    pe->qhat = (R)(sqrt(0.5 * Lr) / mhat);
    pe->a_s = (R)(A * dot(p, eperp));
    pe->a_h = (R)(A * dot(p, epi));
    pe->vs[0] = (R)eperp.x; pe->vs[1] = (R)eperp.y; pe->vs[2] = (R)eperp.z;
    pe->vh[0] = (R)epr.x; pe->vh[1] = (R)epr.y; pe->vh[2] = (R)epr.z;
    pe->refl = 1;
}

// Sphere: lit when theta_R < gT + gR; solve in the T-C-R plane.
template <typename R>
__device__ __forceinline__ bool sphere_refl(const BodyPrep& b, const RxGeo& g, d3 Rp, const LaunchParams& L,
                                            PathEval<R>* pe, PathPts* pts) {
    if (!(b.ok && g.ok)) return false;
    if (!(g.thR - b.gT - g.gR < 0)) return false;
    double th = alhazen(b.a, b.dT, 0.0, g.along, g.wn, g.thR - g.gR, b.gT);
    double s, c;
    sincos(th, &s, &c);
    d3 C = mk(b.c[0], b.c[1], b.c[2]);
    d3 eT = mk(b.eT[0], b.eT[1], b.eT[2]);
    d3 n = c * eT + s * g.eperp;
    d3 Q = C + b.a * n;
    d3 T = mk(L.T[0], L.T[1], L.T[2]);
    if (pts) { pts->P0 = T; pts->P1 = Q; pts->P2 = Q; pts->P3 = Rp; }
    if (pe) refl_common<R>(T, Q, n, Rp, b.a, 2.0 / b.a, 2.0 / b.a, L, pe);
    return true;
}

// Cylinder: lit on the side whose arc is negative; 2-D Alhazen in projection,
// reflection height by proportional split of dz; rho_g = a / cos^2(delta_R).
template <typename R>
__device__ __forceinline__ bool cyl_refl(const BodyPrep& b, const RxGeo& g, d3 Rp, const LaunchParams& L,
                                         PathEval<R>* pe, PathPts* pts) {
    if (!(b.ok && g.ok)) return false;
    double php = g.dphi_plus - b.gT - g.gR;
    double phm = (kTwoPi - g.dphi_plus) - b.gT - g.gR;
    double lo, hi;
    if (php < 0) {
        lo = b.aT + g.dphi_plus - g.gR;
        hi = b.aT + b.gT;
    } else if (phm < 0) {
        lo = b.aT - b.gT;
        hi = b.aT - (kTwoPi - g.dphi_plus) + g.gR;
    } else {
        return false;
    }
    double a = b.a;
    double tx = L.T[0] - b.c[0], ty = L.T[1] - b.c[1];
    double rx = Rp.x - b.c[0], ry = Rp.y - b.c[1];
    double al = alhazen(a, tx, ty, rx, ry, lo, hi);
    double s, c;
    sincos(al, &s, &c);
    double qx = a * c, qy = a * s;
    double lt = sqrt((qx - tx) * (qx - tx) + (qy - ty) * (qy - ty));
    double lr = sqrt((qx - rx) * (qx - rx) + (qy - ry) * (qy - ry));
    double dz = Rp.z - L.T[2];
    double zQ = L.T[2] + dz * lt / (lt + lr);
    if (zQ < b.z0 || zQ > b.z0 + b.h) return false;
    d3 T = mk(L.T[0], L.T[1], L.T[2]);
    d3 Q = mk(b.c[0] + qx, b.c[1] + qy, zQ);
    d3 n = mk(c, s, 0);
    if (pts) { pts->P0 = T; pts->P1 = Q; pts->P2 = Q; pts->P3 = Rp; }
    if (pe) {
        d3 vi = Q - T;
        double sI = norm(vi);
        d3 si = (1.0 / sI) * vi;
        d3 circ = mk(-s, c, 0);
        double sn = dot(si, n);
        d3 tang = si - sn * n;
        double tn2 = dot(tang, tang);
        double tc = dot(tang, circ);
        double cos2d = tn2 > 0 ? tc * tc / tn2 : 1.0;
        if (cos2d < 1e-12) cos2d = 1e-12;
        double cos2b = 1.0 - si.z * si.z;
        refl_common<R>(T, Q, n, Rp, a / cos2d, 2.0 * cos2b / a, 0.0, L, pe);
    }
    return true;
}

}  // namespace utd

// One specular wall bounce (geometric-optics multipath) and the body paths it
// feeds, added to the field of utd_smooth_field when wall reflections are on.
// Included by utd_kernels.hip after the forward kernels.
//
// Reflectors are the planes of the scene triangles: all triangles of one
// plane n.x = d reflect as one mirror (their plane index sits in the w
// component of each triangle's first vertex), and a specular point counts
// when it lies on one of them.  For a planar mirror the reflected wave is
// the wave of the image source T' = T - 2 (n.T - d) n, so with one bounce a
// receiver R gets (the equivalent source of Fig. 1 feeding the
// surface-diffracted paths of Eqs. (2)-(4)):
//   wall only   T -> Q_w -> R              (lit branch on)
//   wall, body  T -> Q_w -> body -> R      T' as the source of the body's two
//                                          primary creeping paths and its
//                                          reflection (lit branch on)
//   body, wall  T -> body -> Q_w -> R      the same towards the image
//                                          receiver R' of R
// The wall maps the incident polarisation v on the ray direction s_in to
// R_perp (v.e_perp) e_perp + R_par (v.e_par_in) e_par_out (e_perp = s_in x n
// normalised, e_par = e_perp x s); R_perp, R_par are the plane-wave
// coefficients of a homogeneous slab (or -1, +1 for a perfect conductor).
// Because they are frequency dependent and the map mixes polarisations, a
// body path fed by (or feeding) a wall is evaluated as two paths with fixed
// polarisation vectors, A (the perpendicular part) and B (the parallel
// part), sharing one Fock evaluation per frequency:
//   E += R_perp(f) E_A(f) + R_par(f) E_B(f).
//
// k_walls_prep  body constants of every (plane, body) for the image source
// k_walls       one lane per receiver: every plane, then every body, with the
//               visibility of each leg tested on the spot (BVH any-hit with a
//               per-lane LDS stack, body tests), and the field of each
//               visible path added to E at every frequency.
#pragma once

namespace utd {

constexpr double kEps0 = 8.8541878128e-12;

// Slab reflection coefficients at incidence cosine ct and frequency f, FP64:
// eta = eps_r - j sigma / (w eps0), c = sqrt(eta - sin^2) with Im c <= 0,
// r_perp = (ct - c)/(ct + c), r_par = (eta ct - c)/(eta ct + c), and with the
// internal round trip ph = e^{-2 j k t c}: R = r (1 - ph) / (1 - r^2 ph).
__device__ __forceinline__ void slab_coef(double ct, double f, const WallMat& m, cplx<double>* rp,
                                          cplx<double>* rl) {
    if (m.pec) {
        *rp = cplx<double>{-1.0, 0.0};
        *rl = cplx<double>{1.0, 0.0};
        return;
    }
    const double w = kTwoPi * f;
    const cplx<double> eta{m.eps_r, -m.sigma / (w * kEps0)};
    const double x = eta.re - (1.0 - ct * ct), y = eta.im;
    const double r = sqrt(x * x + y * y);
    const cplx<double> c{sqrt(fmax(0.5 * (r + x), 0.0)), -sqrt(fmax(0.5 * (r - x), 0.0))};
    auto cdiv = [](cplx<double> a, cplx<double> b) {
        const double id = 1.0 / (b.re * b.re + b.im * b.im);
        return cplx<double>{(a.re * b.re + a.im * b.im) * id, (a.im * b.re - a.re * b.im) * id};
    };
    const cplx<double> ec{eta.re * ct, eta.im * ct};
    cplx<double> a = cdiv(cplx<double>{ct - c.re, -c.im}, cplx<double>{ct + c.re, c.im});
    cplx<double> b = cdiv(cplx<double>{ec.re - c.re, ec.im - c.im}, cplx<double>{ec.re + c.re, ec.im + c.im});
    if (isfinite(m.thickness)) {
        // ph = e^{-2 j k t c} = e^{2 k t Im c} e^{-2 j k t Re c}
        const double kt2 = 2.0 * (w / kC0) * m.thickness;
        double sn, cs;
        sincos(kt2 * c.re, &sn, &cs);
        const double mag = exp(kt2 * c.im);
        const cplx<double> ph{mag * cs, -mag * sn};
        auto slab = [&](cplx<double> q) {
            const cplx<double> num = cmul(q, cplx<double>{1.0 - ph.re, -ph.im});
            const cplx<double> q2ph = cmul(cmul(q, q), ph);
            return cdiv(num, cplx<double>{1.0 - q2ph.re, -q2ph.im});
        };
        a = slab(a);
        b = slab(b);
    }
    *rp = a;
    *rl = b;
}

// (e_perp, e_par_in, e_par_out, cos) of a reflection on a plane of normal n.
struct WallBasis {
    d3 ep, ei, eo;
    double ct;
};
__device__ __forceinline__ WallBasis wall_basis(d3 s_in, d3 s_out, d3 n) {
    WallBasis w;
    d3 c = cross(s_in, n);
    const double cn = norm(c);
    w.ep = cn > 1e-12 ? (1.0 / cn) * c : any_perp(n);
    w.ei = cross(w.ep, s_in);
    w.eo = cross(w.ep, s_out);
    w.ct = fabs(dot(s_in, n));
    return w;
}

__device__ __forceinline__ d3 unit3(d3 v) { return (1.0 / norm(v)) * v; }

// Where the segment A -> B crosses the plane strictly between its end
// points (heights ha, hb of A and B above the plane): false if it does not.
__device__ __forceinline__ bool plane_crossing(d3 A, d3 B, double ha, double hb, d3* Q) {
    if (!((ha > 0.0 && hb < 0.0) || (ha < 0.0 && hb > 0.0))) return false;
    const double t = ha / (ha - hb);
    *Q = A + t * (B - A);
    return true;
}

// Triangle test restricted to the triangles of one plane (index in the w
// component of each triangle's first vertex).
__device__ __forceinline__ bool bvh_anyhit_plane(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                                 const SegRay& r, int* stack, int stride, int root, int plane) {
    int sp = 0;
    int node = root;
    for (;;) {
        float4 q0 = nodes[4 * node + 0];
        float4 q1 = nodes[4 * node + 1];
        float4 q2 = nodes[4 * node + 2];
        int4 q3 = *reinterpret_cast<const int4*>(&nodes[4 * node + 3]);
        bool h0 = q3.x >= 0 && box_hit(r, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y);
        bool h1 = q3.z >= 0 && box_hit(r, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w);
        int next = -1;
        if (h0) {
            if (q3.y > 0) {
                for (int t = q3.x; t < q3.x + q3.y; ++t) {
                    const float4 a = tris[3 * t];
                    if (__float_as_int(a.w) == plane && tri_hit(r, a, tris[3 * t + 1], tris[3 * t + 2])) return true;
                }
            } else {
                next = q3.x;
            }
        }
        if (h1) {
            if (q3.w > 0) {
                for (int t = q3.z; t < q3.z + q3.w; ++t) {
                    const float4 a = tris[3 * t];
                    if (__float_as_int(a.w) == plane && tri_hit(r, a, tris[3 * t + 1], tris[3 * t + 2])) return true;
                }
            } else if (next < 0) {
                next = q3.z;
            } else if (sp < kStackDepth) {
                stack[stride * sp++] = q3.z;
            }
        }
        if (next >= 0) {
            node = next;
        } else if (sp > 0) {
            node = stack[stride * --sp];
        } else {
            return false;
        }
    }
}

// Does the point Q of plane p lie on one of the plane's triangles?  A short
// segment through Q along the normal, against that plane's triangles in both
// trees; the plane's bounding box first.
__device__ __forceinline__ bool on_reflector(const WallPlane& P, int p, d3 Q, const LaunchParams& L,
                                             const float4* nodes, const float4* tris, int* stk, int stride) {
    const double sl = 1e-6;
    if (Q.x < P.lo[0] - sl || Q.x > P.hi[0] + sl || Q.y < P.lo[1] - sl || Q.y > P.hi[1] + sl ||
        Q.z < P.lo[2] - sl || Q.z > P.hi[2] + sl)
        return false;
    const d3 n = mk(P.n[0], P.n[1], P.n[2]);
    const SegRay r = make_ray(Q - 1e-3 * n, Q + 1e-3 * n);
    if (bvh_anyhit_plane(nodes, tris, r, stk, stride, 0, p)) return true;
    return L.broot >= 0 && bvh_anyhit_plane(nodes, tris, r, stk, stride, L.broot, p);
}

// Body constants of every (plane, body) pair for the plane's image source.
__global__ void __launch_bounds__(256) k_walls_prep(LaunchParams L, const float* __restrict__ sph,
                                                    const float* __restrict__ cyl, const WallPlane* __restrict__ planes,
                                                    int n_planes, BodyPrep* __restrict__ prep_img) {
    const int nb = L.n_sph + L.n_cyl;
    const int64_t n = (int64_t)n_planes * nb;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(k / nb), b = (int)(k % nb);
        const WallPlane P = planes[p];
        const double h = P.n[0] * L.T[0] + P.n[1] * L.T[1] + P.n[2] * L.T[2] - P.d;
        double Ti[3] = {L.T[0] - 2.0 * h * P.n[0], L.T[1] - 2.0 * h * P.n[1], L.T[2] - 2.0 * h * P.n[2]};
        prep_img[k] = body_prep(Ti, sph, L.n_sph, cyl, b);
    }
}

// One wall-bounce body path at one frequency: the Fock coefficients once,
// the two polarisation parts weighted by the wall coefficients.
template <typename R, int MODE>
__device__ __forceinline__ void add_wall_body(const PathEval<R>& pe, const R vsB[3], const R vhB[3],
                                              const Tabs<R>& tb, const FreqC<R>& fc, cplx<R> rp, cplx<R> rl,
                                              R* E) {
    FockArgs<R> a;
    a.xi = fc.k13 * pe.xh;
    a.u = fc.sk * pe.uh;
    a.iu = fc.isk * pe.iuh;
    a.ixi = fc.ik13 * pe.ixh;
    a.h = (R)0.5 * fc.k16 * pe.sxh;
    a.qc = fc.k16 * (pe.qhat * (R)-kC2E4);
    a.xc = fc.ik13 * (pe.ixh * (R)kC2E4);
    cplx<R> Ks, Kh;
    fock_kernel<R, MODE>(tb, a, pe.refl != 0, &Ks, &Kh);
    cplx<R> ph = phase_rev<R>(fc.rev_per_m * pe.s_tot - 0.25 * pe.nc);
    ph.re *= fc.km16;
    ph.im *= fc.km16;
    const cplx<R> cs = cmul(Ks, ph), ch = cmul(Kh, ph);
    // A part times R_perp, B part times R_par
    const cplx<R> ps = cmul(cs, rp), phA = cmul(ch, rp), qs = cmul(cs, rl), qh = cmul(ch, rl);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        E[2 * c] += ps.re * pe.vs[c] + phA.re * pe.vh[c] + qs.re * vsB[c] + qh.re * vhB[c];
        E[2 * c + 1] += ps.im * pe.vs[c] + phA.im * pe.vh[c] + qs.im * vsB[c] + qh.im * vhB[c];
    }
}

// Splits the output polarisation vectors of a body path reaching the wall
// into the parts the wall reflects with R_perp (kept in pe) and R_par (out).
template <typename R>
__device__ __forceinline__ void split_out(const WallBasis& w, PathEval<R>* pe, R vsB[3], R vhB[3]) {
    const R epx = (R)w.ep.x, epy = (R)w.ep.y, epz = (R)w.ep.z;
    const R eix = (R)w.ei.x, eiy = (R)w.ei.y, eiz = (R)w.ei.z;
    const R eox = (R)w.eo.x, eoy = (R)w.eo.y, eoz = (R)w.eo.z;
    const R sa = pe->vs[0] * epx + pe->vs[1] * epy + pe->vs[2] * epz;
    const R sb = pe->vs[0] * eix + pe->vs[1] * eiy + pe->vs[2] * eiz;
    const R ha = pe->vh[0] * epx + pe->vh[1] * epy + pe->vh[2] * epz;
    const R hb = pe->vh[0] * eix + pe->vh[1] * eiy + pe->vh[2] * eiz;
    vsB[0] = sb * eox; vsB[1] = sb * eoy; vsB[2] = sb * eoz;
    vhB[0] = hb * eox; vhB[1] = hb * eoy; vhB[2] = hb * eoz;
    pe->vs[0] = sa * epx; pe->vs[1] = sa * epy; pe->vs[2] = sa * epz;
    pe->vh[0] = ha * epx; pe->vh[1] = ha * epy; pe->vh[2] = ha * epz;
}

// Wall-decision bits per (receiver, plane): bit 0 the wall-only path; body b
// takes bits 1 + 6 b + k, k = 0/1 wall then creeping side +/-, 2 wall then
// reflection, 3/4 creeping side +/- then wall, 5 reflection then wall.
constexpr int kWallMaskBodies = 10;

template <typename R>
__global__ void __launch_bounds__(256) k_walls(LaunchParams L, WallMat M, const float* __restrict__ rx,
                                               const float* __restrict__ sph, const float* __restrict__ cyl,
                                               const BodyPrep* __restrict__ prep,
                                               const BodyPrep* __restrict__ prep_img,
                                               const WallPlane* __restrict__ planes, int n_planes,
                                               const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                               const FreqConst* __restrict__ fcs, const double* __restrict__ freqs,
                                               uint8_t* __restrict__ flags, R* __restrict__ E_out,
                                               uint64_t* __restrict__ wmask) {
    __shared__ __attribute__((aligned(16))) R s_reg[TableStage<R>::NREG];
    __shared__ __attribute__((aligned(16))) R s_tf[TableStage<R>::NTF];
    __shared__ int stack[kStackDepth * 256];
    const Tabs<R> tb = TableStage<R>::template stage<256>(s_reg, s_tf);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n_rx) return;
    int* stk = stack + threadIdx.x;
    const uint8_t fl = flags[i];
    const bool dead = (fl & kFlagDead) != 0;
    const d3 T = mk(L.T[0], L.T[1], L.T[2]);
    const d3 R3 = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
    const int nb = L.n_sph + L.n_cyl;
    const bool bo = L.bodies_occlude != 0;
    bool caus = false;
    auto add_all_freqs = [&](auto&& one) {
        for (int j = 0; j < L.n_f; ++j) {
            if (!fcs[j].ok) continue;
            R e[6];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int64_t o = ((int64_t)j * 3 + c) * L.n_rx + i;
                e[2 * c] = E_out[2 * o];
                e[2 * c + 1] = E_out[2 * o + 1];
            }
            one(j, e);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int64_t o = ((int64_t)j * 3 + c) * L.n_rx + i;
                E_out[2 * o] = e[2 * c];
                E_out[2 * o + 1] = e[2 * c + 1];
            }
        }
    };
    for (int p = 0; p < n_planes; ++p) {
        uint64_t bits = 0;
        const WallPlane P = planes[p];
        const d3 n = mk(P.n[0], P.n[1], P.n[2]);
        const double hT = dot(n, T) - P.d;
        if (dead || hT == 0.0) {
            if (wmask) wmask[i * n_planes + p] = 0;
            continue;
        }
        const d3 Ti = T - (2.0 * hT) * n;
        const double hR = dot(n, R3) - P.d;
        // --- wall only ---------------------------------------------------------
        d3 Qw;
        if (L.lit_branch && plane_crossing(Ti, R3, -hT, hR, &Qw) && on_reflector(P, p, Qw, L, nodes, tris, stk, 256) &&
            !seg_blocked(T, Qw, L, sph, cyl, -1, true, nodes, tris, stk, 256) &&
            !seg_blocked(Qw, R3, L, sph, cyl, -1, true, nodes, tris, stk, 256)) {
            bits |= 1ull;
            const d3 si = Qw - T, sr = R3 - Qw;
            const double li = norm(si), lr = norm(sr);
            const WallBasis w = wall_basis((1.0 / li) * si, (1.0 / lr) * sr, n);
            const d3 sh = (1.0 / li) * si;
            const d3 pv = mk(L.p[0], L.p[1], L.p[2]);
            const d3 pp = L.amp * (pv - dot(pv, sh) * sh);
            const double a = dot(pp, w.ep), b = dot(pp, w.ei);
            const double s = li + lr, is = 1.0 / s;
            add_all_freqs([&](int j, R* e) {
                cplx<double> rp, rl;
                slab_coef(w.ct, freqs[j], M, &rp, &rl);
                const cplx<R> ph = phase_rev<R>(fcs[j].rev_per_m * s);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double ep = c == 0 ? w.ep.x : (c == 1 ? w.ep.y : w.ep.z);
                    const double eo = c == 0 ? w.eo.x : (c == 1 ? w.eo.y : w.eo.z);
                    const R vre = (R)(is * (a * rp.re * ep + b * rl.re * eo));
                    const R vim = (R)(is * (a * rp.im * ep + b * rl.im * eo));
                    e[2 * c] += vre * ph.re - vim * ph.im;
                    e[2 * c + 1] += vre * ph.im + vim * ph.re;
                }
            });
        }
        // --- bodies ------------------------------------------------------------
        const d3 Ri = R3 - (2.0 * hR) * n;
        for (int b = 0; b < nb; ++b) {
            // wall then body: the image source T' feeds the body
            const BodyPrep Pi = prep_img[(int64_t)p * nb + b];
            if (Pi.ok && (Pi.kind == 0 || cyl_paths_possible(Pi, R3, Ti, L))) {
                const RxGeo g = rx_geo(Pi, R3);
                for (int k = 0; k < 3; ++k) {
                    if (k == 2 && !L.lit_branch) break;
                    PathPts pts;
                    double th = 0.0;
                    bool ok;
                    d3 Qb, nb3;
                    if (k < 2) {
                        bool cz = false;
                        const int sgn = k == 0 ? 1 : -1;
                        ok = Pi.kind == 0 ? sphere_creep<R, double>(Pi, g, R3, Ti, L, sgn, 0, &cz, (PathEval<R>*)nullptr, &pts)
                                          : cyl_creep<R, double>(Pi, g, R3, Ti, L, sgn, 0, (PathEval<R>*)nullptr, &pts);
                        caus |= cz;
                    } else {
                        ok = refl_angle<Kinds::Any, (sizeof(R) == 8)>(Pi, g, R3, Ti, &th);
                        if (ok) {
                            refl_point<double>(Pi, g, R3, Ti, th, &Qb, &nb3);
                            pts.P1 = Qb; pts.P2 = Qb;
                        }
                    }
                    if (!ok) continue;
                    const d3 Qin = pts.P1, Qout = pts.P2;
                    if (!plane_crossing(Ti, Qin, -hT, dot(n, Qin) - P.d, &Qw)) continue;
                    if (!on_reflector(P, p, Qw, L, nodes, tris, stk, 256)) continue;
                    if (seg_blocked(T, Qw, L, sph, cyl, -1, bo, nodes, tris, stk, 256) ||
                        seg_blocked(Qw, Qin, L, sph, cyl, b, bo, nodes, tris, stk, 256) ||
                        seg_blocked(Qout, R3, L, sph, cyl, b, bo, nodes, tris, stk, 256))
                        continue;
                    if (b < kWallMaskBodies) bits |= 1ull << (1 + 6 * b + k);
                    // incident polarisation at the body after the wall: the A
                    // (perpendicular) and B (parallel) parts as the "dipole"
                    const d3 sh = unit3(Qw - T);
                    const WallBasis w = wall_basis(sh, unit3(Qin - Qw), n);
                    const d3 pv = mk(L.p[0], L.p[1], L.p[2]);
                    const d3 pp = pv - dot(pv, sh) * sh;
                    const d3 uA = dot(pp, w.ep) * w.ep, uB = dot(pp, w.ei) * w.eo;
                    LaunchParams LA = L, LB = L;
                    LA.p[0] = uA.x; LA.p[1] = uA.y; LA.p[2] = uA.z;
                    LB.p[0] = uB.x; LB.p[1] = uB.y; LB.p[2] = uB.z;
                    PathEval<R> pA, pB;
                    if (k < 2) {
                        bool cz;
                        const int sgn = k == 0 ? 1 : -1;
                        if (Pi.kind == 0) {
                            sphere_creep<R, double>(Pi, g, R3, Ti, LA, sgn, 0, &cz, &pA, nullptr);
                            sphere_creep<R, double>(Pi, g, R3, Ti, LB, sgn, 0, &cz, &pB, nullptr);
                        } else {
                            cyl_creep<R, double>(Pi, g, R3, Ti, LA, sgn, 0, &pA, nullptr);
                            cyl_creep<R, double>(Pi, g, R3, Ti, LB, sgn, 0, &pB, nullptr);
                        }
                    } else {
                        refl_eval<R, double>(Pi, Qb, nb3, R3, Ti, LA, &pA);
                        refl_eval<R, double>(Pi, Qb, nb3, R3, Ti, LB, &pB);
                    }
                    const double ct = w.ct;
                    add_all_freqs([&](int j, R* e) {
                        cplx<double> rp, rl;
                        slab_coef(ct, freqs[j], M, &rp, &rl);
                        const FreqC<R> fc(fcs[j]);
                        if (k < 2)
                            add_wall_body<R, kCreep>(pA, pB.vs, pB.vh, tb, fc, cplx<R>{(R)rp.re, (R)rp.im},
                                                     cplx<R>{(R)rl.re, (R)rl.im}, e);
                        else
                            add_wall_body<R, kRefl>(pA, pB.vs, pB.vh, tb, fc, cplx<R>{(R)rp.re, (R)rp.im},
                                                    cplx<R>{(R)rl.re, (R)rl.im}, e);
                    });
                }
            }
            // body then wall: the body's paths towards the image receiver R'
            const BodyPrep P0 = prep[b];
            if (P0.ok && (P0.kind == 0 || cyl_paths_possible(P0, Ri, T, L))) {
                const RxGeo g = rx_geo(P0, Ri);
                for (int k = 0; k < 3; ++k) {
                    if (k == 2 && !L.lit_branch) break;
                    PathPts pts;
                    double th = 0.0;
                    bool ok;
                    d3 Qb, nb3;
                    if (k < 2) {
                        bool cz = false;
                        const int sgn = k == 0 ? 1 : -1;
                        ok = P0.kind == 0 ? sphere_creep<R, double>(P0, g, Ri, T, L, sgn, 0, &cz, (PathEval<R>*)nullptr, &pts)
                                          : cyl_creep<R, double>(P0, g, Ri, T, L, sgn, 0, (PathEval<R>*)nullptr, &pts);
                        caus |= cz;
                    } else {
                        ok = refl_angle<Kinds::Any, (sizeof(R) == 8)>(P0, g, Ri, T, &th);
                        if (ok) {
                            refl_point<double>(P0, g, Ri, T, th, &Qb, &nb3);
                            pts.P1 = Qb; pts.P2 = Qb;
                        }
                    }
                    if (!ok) continue;
                    const d3 Qin = pts.P1, Qout = pts.P2;
                    if (!plane_crossing(Qout, Ri, dot(n, Qout) - P.d, -hR, &Qw)) continue;
                    if (!on_reflector(P, p, Qw, L, nodes, tris, stk, 256)) continue;
                    if (seg_blocked(T, Qin, L, sph, cyl, b, bo, nodes, tris, stk, 256) ||
                        seg_blocked(Qout, Qw, L, sph, cyl, b, bo, nodes, tris, stk, 256) ||
                        seg_blocked(Qw, R3, L, sph, cyl, -1, bo, nodes, tris, stk, 256))
                        continue;
                    if (b < kWallMaskBodies) bits |= 1ull << (1 + 6 * b + 3 + k);
                    PathEval<R> pA;
                    if (k < 2) {
                        bool cz;
                        const int sgn = k == 0 ? 1 : -1;
                        if (P0.kind == 0)
                            sphere_creep<R, double>(P0, g, Ri, T, L, sgn, 0, &cz, &pA, nullptr);
                        else
                            cyl_creep<R, double>(P0, g, Ri, T, L, sgn, 0, &pA, nullptr);
                    } else {
                        refl_eval<R, double>(P0, Qb, nb3, Ri, T, L, &pA);
                    }
                    const WallBasis w = wall_basis(unit3(Qw - Qout), unit3(R3 - Qw), n);
                    R vsB[3], vhB[3];
                    split_out<R>(w, &pA, vsB, vhB);
                    const double ct = w.ct;
                    add_all_freqs([&](int j, R* e) {
                        cplx<double> rp, rl;
                        slab_coef(ct, freqs[j], M, &rp, &rl);
                        const FreqC<R> fc(fcs[j]);
                        if (k < 2)
                            add_wall_body<R, kCreep>(pA, vsB, vhB, tb, fc, cplx<R>{(R)rp.re, (R)rp.im},
                                                     cplx<R>{(R)rl.re, (R)rl.im}, e);
                        else
                            add_wall_body<R, kRefl>(pA, vsB, vhB, tb, fc, cplx<R>{(R)rp.re, (R)rp.im},
                                                    cplx<R>{(R)rl.re, (R)rl.im}, e);
                    });
                }
            }
        }
        if (wmask) wmask[i * n_planes + p] = bits;
    }
    if (caus) flags[i] = (uint8_t)(flags[i] | kFlagCaustic);
}

}  // namespace utd

namespace utd {

size_t walls_scratch_bytes(const LaunchParams& L, int n_planes) {
    return sizeof(BodyPrep) * (size_t)n_planes * (size_t)(L.n_sph + L.n_cyl > 0 ? L.n_sph + L.n_cyl : 1);
}

template <typename R>
static hipError_t launch_walls_t(const LaunchParams& L, const WallMat& M, const float* rx, const float* sph,
                                 const float* cyl, const BodyPrep* prep, BodyPrep* prep_img, const WallPlane* planes,
                                 int n_planes, const float4* nodes, const float4* tris, const FreqConst* fcs,
                                 const double* freqs, uint8_t* flags, R* E, uint64_t* wmask, hipStream_t s) {
    const int nb = L.n_sph + L.n_cyl;
    hipError_t e;
    if (nb > 0) {
        const int64_t n = (int64_t)n_planes * nb;
        const int64_t g = (n + 255) / 256;
        hipLaunchKernelGGL(k_walls_prep, dim3((unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g))), dim3(256), 0, s, L, sph,
                           cyl, planes, n_planes, prep_img);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_walls<R>), dim3((unsigned)((L.n_rx + 255) / 256)), dim3(256), 0, s, L, M, rx, sph, cyl, prep,
                       prep_img, planes, n_planes, nodes, tris, fcs, freqs, flags, E, wmask);
    return hipGetLastError();
}

hipError_t launch_walls(const LaunchParams& L, int precision, const WallMat& M, const float* rx, const float* sph,
                        const float* cyl, const BodyPrep* prep, BodyPrep* prep_img, const WallPlane* planes,
                        int n_planes, const float4* nodes, const float4* tris, const FreqConst* fcs,
                        const double* freqs, uint8_t* flags, void* E, uint64_t* wmask, hipStream_t s) {
    if (L.n_rx == 0 || n_planes == 0) return hipSuccess;
    return precision == 0 ? launch_walls_t<float>(L, M, rx, sph, cyl, prep, prep_img, planes, n_planes, nodes, tris,
                                                  fcs, freqs, flags, (float*)E, wmask, s)
                          : launch_walls_t<double>(L, M, rx, sph, cyl, prep, prep_img, planes, n_planes, nodes, tris,
                                                   fcs, freqs, flags, (double*)E, wmask, s);
}

}  // namespace utd

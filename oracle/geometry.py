"""Ray geometry on PEC spheres and vertical PEC cylinders, FP64.

Test infrastructure (see ``oracle/__init__``).

For one body and many receivers (vectorised over receivers) this returns the
frequency-independent description of every ray path the UTD sums:

* creeping paths (Eq. (4)): attachment point Q1 on the shadow boundary seen
  from the source, geodesic Q1 -> Q2 on the surface, detachment point Q2 on
  the shadow boundary seen from the receiver; one path on each side of the
  body plus ``l_enc`` extra encirclements (the generalised Fermat principle
  of Sec. III-B);
* the specular reflection (Eq. (3)) when the receiver is lit.

Frames: n is the outward normal, t the direction of propagation and
b = t x n.  Spreading factors follow from the ray-tube geometry; they are
written out in ``sphere_creeping`` and ``cylinder_creeping``.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def _norm(v):
    return np.sqrt(np.einsum("...i,...i->...", v, v))


def _unit(v):
    return v / _norm(v)[..., None]


def _any_perp(e):
    """A unit vector perpendicular to each row of e (used only when the
    source, the centre and the receiver are collinear)."""
    ref = np.where(np.abs(e[..., 0:1]) < 0.9, np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]))
    return _unit(np.cross(e, ref))


# ---------------------------------------------------------------------------
# Sphere
# ---------------------------------------------------------------------------


def sphere_frame(T, C, a, R):
    """Per receiver: the plane basis (e_T, e_perp) of the plane through source
    T, centre C and receiver R, with R at polar angle theta_R in [0, pi]."""
    dT = _norm(T - C)
    eT = (T - C) / dT
    v = R - C
    dR = _norm(v)
    along = v @ eT
    w = v - along[:, None] * eT[None, :]
    wn = _norm(w)
    # on the axis (the plane of T, C and R undefined; w is rounding noise
    # below a relative 1e-12) any perpendicular serves
    on_axis = wn <= 1e-12 * dR
    eperp = np.where(on_axis[:, None], _any_perp(np.broadcast_to(eT, v.shape)),
                     w / np.where(on_axis, 1.0, wn)[:, None])
    wn = np.where(on_axis, 0.0, wn)
    thR = np.arctan2(wn, along)
    return dT, eT, dR, eperp, thR


def sphere_creeping(T, C, a, R, side, ell):
    """Creeping path on side ``side`` (+1 or -1) with ``ell`` encirclements.

    Side +1 leaves the source's tangent cone towards the receiver's half of
    the T-C-R plane, side -1 goes around the far side.  With
    gamma_T = acos(a/d_T), gamma_R = acos(a/d_R):
        phi_+ = theta_R - gamma_T - gamma_R + 2 pi ell
        phi_- = 2 pi - theta_R - gamma_T - gamma_R + 2 pi ell
    and the path exists when phi >= 0.  The geodesic is the great circle in
    the T-C-R plane; with theta2 = gamma_T + phi the polar angle of Q2,

        dη(Q1)/dη(Q2) = sin(gamma_T)/sin(theta2)   (meridians through the pole e_T)
        rho^d         = a tan(theta2)               (shed rays meet the axis)

    so that sqrt(dη1/dη2) sqrt(rho^d / (s^d (rho^d + s^d))) has modulus
    sqrt(a sin(gamma_T) / (s^d |rho_perp|)) with rho_perp = a sin theta2 + s^d cos theta2
    the signed distance of R from the source axis.  Each caustic passed adds
    +pi/2 (e^{+jwt}): floor(theta2/pi) surface poles plus one more when the
    shed ray crosses the axis before R.
    """
    dT, eT, dR, eperp, thR = sphere_frame(T, C, a, R)
    sI = np.sqrt(dT * dT - a * a)
    sD = np.sqrt(np.maximum(dR * dR - a * a, 0.0))
    gT = np.arctan2(sI, a)
    gR = np.arctan2(sD, a)
    if side > 0:
        phi = thR - gT - gR + TWO_PI * ell
        ep = eperp
    else:
        phi = TWO_PI - thR - gT - gR + TWO_PI * ell
        ep = -eperp
    th2 = gT + phi
    c1, s1 = np.cos(gT), np.sin(gT)
    c2, s2 = np.cos(th2), np.sin(th2)
    eTb = np.broadcast_to(eT, R.shape)
    n1 = c1 * eTb + s1 * ep
    t1 = -s1 * eTb + c1 * ep
    n2 = c2[:, None] * eTb + s2[:, None] * ep
    t2 = -s2[:, None] * eTb + c2[:, None] * ep
    b = np.cross(t1, n1)
    Q1 = C + a * n1
    Q2 = C + a * n2
    # signed distance of R from the source axis: a sin th2 + s^d cos th2,
    # whose magnitude is d_R sin theta_R; the sum cancels near the axis
    # (an absolute error of ~1e-15 m), so only its sign is taken from it
    rho_perp = np.sign(a * s2 + sD * c2) * (dR * np.sin(thR))
    Nc = np.floor(th2 / np.pi) + (np.sign(rho_perp) != np.sign(s2))
    amp = np.sqrt(a * s1 / (sD * np.abs(rho_perp)))
    S = amp * np.exp(0.5j * np.pi * Nc)
    t = a * phi
    return dict(kind="creep", valid=phi >= 0, phi=phi, Q1=Q1, Q2=Q2,
                n1=n1, b1=b, n2=n2, b2=b, t1=t1, t2=t2,
                s_i=np.broadcast_to(sI, phi.shape), t=t, s_d=sD,
                rho_g=np.full(phi.shape, a), S=S, rho_perp=rho_perp)


def _bisect_stationary(g, lo, hi, iters=100):
    """Root of g on [lo, hi] (vectorised) given a sign change; bisection."""
    glo = g(lo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        gm = g(mid)
        same = np.sign(gm) == np.sign(glo)
        lo = np.where(same, mid, lo)
        glo = np.where(same, gm, glo)
        hi = np.where(same, hi, mid)
    return 0.5 * (lo + hi)


def sphere_reflection(T, C, a, R):
    """Specular point on the sphere for lit receivers (phi_+ < 0).

    Alhazen's problem in the T-C-R plane: the point Q = a(cos th, sin th) of
    the arc seen from both T and R, th in [theta_R - gamma_R, gamma_T], at
    which d/dth (|Q - T| + |Q - R|) = 0, found by bisection in FP64.
    Caustic distances of the reflected wave for a point source on a sphere
    (Kouyoumjian and Pathak 1974):
        1/rho_1 = 1/s^i + 2/(a cos th_i),   1/rho_2 = 1/s^i + 2 cos th_i / a
    with rho_1 in the plane of incidence.  The radius of curvature in the
    plane of incidence is rho_g = a.
    """
    dT, eT, dR, eperp, thR = sphere_frame(T, C, a, R)
    sI0 = np.sqrt(dT * dT - a * a)
    sD0 = np.sqrt(np.maximum(dR * dR - a * a, 0.0))
    gT = np.arctan2(sI0, a)
    gR = np.arctan2(sD0, a)
    lit = thR - gT - gR < 0
    Tx, Ty = dT, 0.0
    Rx, Ry = dR * np.cos(thR), dR * np.sin(thR)

    def g(th):
        qx, qy = a * np.cos(th), a * np.sin(th)
        tx, ty = -np.sin(th), np.cos(th)
        dt = np.hypot(qx - Tx, qy - Ty)
        dr = np.hypot(qx - Rx, qy - Ry)
        return ((qx - Tx) * tx + (qy - Ty) * ty) / dt + ((qx - Rx) * tx + (qy - Ry) * ty) / dr

    lo = np.where(lit, thR - gR, 0.0)
    hi = np.where(lit, np.broadcast_to(gT, thR.shape), 1.0)
    th = _bisect_stationary(g, lo, hi)
    eTb = np.broadcast_to(eT, R.shape)
    n = np.cos(th)[:, None] * eTb + np.sin(th)[:, None] * eperp
    Q = C + a * n
    return _reflection_common(T, R, Q, n, lit, rho_g=np.full(th.shape, a),
                              inv_f1_cos=np.full(th.shape, 2.0 / a),
                              inv_f2_over_cos=np.full(th.shape, 2.0 / a))


def _reflection_common(T, R, Q, n, valid, rho_g, inv_f1_cos, inv_f2_over_cos):
    """Shared reflection bookkeeping.

    The reflected-wave caustic distances are written as
        1/rho_1 = 1/s^i + inv_f1_cos / cos th_i,   1/rho_2 = 1/s^i + inv_f2_over_cos * cos th_i
    so that rho_1/cos th_i = 1/(cos th_i/s^i + inv_f1_cos) stays finite at
    grazing incidence.
    """
    vi = Q - T
    sI = _norm(vi)
    si_hat = vi / sI[:, None]
    vr = R - Q
    sR = _norm(vr)
    sr_hat = vr / sR[:, None]
    cos_i = -np.einsum("ij,ij->i", si_hat, n)
    cos_i = np.clip(cos_i, 0.0, 1.0)
    rho1_over_cos = 1.0 / (cos_i / sI + inv_f1_cos)
    rho1 = rho1_over_cos * cos_i
    inv_rho2 = 1.0 / sI + inv_f2_over_cos * cos_i
    rho2 = 1.0 / inv_rho2
    cr = np.cross(si_hat, n)
    crn = _norm(cr)
    # at normal incidence the plane of incidence is undefined, and on a
    # curved surface R_s != -R_h, so the field depends on the basis chosen:
    # within sin(th_i) <= 1e-6 (the resolution of an FP32 frame) the fixed
    # perpendicular of n is taken
    eperp = np.where((crn > 1e-6)[:, None], cr / np.maximum(crn, 1e-300)[:, None], _any_perp(n))
    epar_i = np.cross(eperp, si_hat)
    epar_r = np.cross(eperp, sr_hat)
    return dict(kind="refl", valid=valid, Q=Q, n=n, s_i=sI, s_r=sR, si_hat=si_hat, sr_hat=sr_hat,
                cos_i=cos_i, rho1_over_cos=rho1_over_cos, rho1=rho1, rho2=rho2,
                rho_g=rho_g, eperp=eperp, epar_i=epar_i, epar_r=epar_r)


# ---------------------------------------------------------------------------
# Vertical cylinder (axis parallel to z, lateral surface z in [z0, z0 + h])
# ---------------------------------------------------------------------------


def cylinder_plan(T, cyl, R):
    """Projected (xy) geometry: distances to the axis, tangent half-angles,
    tangent lengths and the CCW angle from T to R around the axis."""
    cx, cy, z0, h, a = cyl
    Tp = np.array([T[0] - cx, T[1] - cy])
    Rp = np.stack([R[:, 0] - cx, R[:, 1] - cy], axis=1)
    rhoT = np.hypot(*Tp)
    rhoR = np.hypot(Rp[:, 0], Rp[:, 1])
    dT = np.sqrt(max(rhoT * rhoT - a * a, 0.0))
    dR = np.sqrt(np.maximum(rhoR * rhoR - a * a, 0.0))
    gT = np.arctan2(dT, a)
    gR = np.arctan2(dR, a)
    aT = np.arctan2(Tp[1], Tp[0])
    aR = np.arctan2(Rp[:, 1], Rp[:, 0])
    dphi_plus = np.mod(aR - aT, TWO_PI)
    return dict(rhoT=rhoT, rhoR=rhoR, dT=dT, dR=dR, gT=gT, gR=gR, aT=aT, aR=aR,
                dphi_plus=dphi_plus)


def cylinder_creeping(T, cyl, R, side, ell, plan=None):
    """Helical creeping path on a vertical cylinder.

    In projection the path is: tangent from T, arc of a*phi around the
    circle, tangent to R, with phi = dphi_side - gamma_T - gamma_R + 2 pi ell
    (dphi_+ CCW from T to R, dphi_- = 2 pi - dphi_+).  Unrolled, the surface
    is a plane and the geodesic a straight line, so the path rises uniformly:
    with L2 = d_T + a phi + d_R and dz = R_z - T_z,
        cos(delta) = L2 / sqrt(L2^2 + dz^2),  s^i = d_T/cos, t = a phi/cos, s^d = d_R/cos.
    The radius of curvature along the helix is rho_g = a / cos^2(delta).
    Spreading: in the developed tangent plane the surface rays fan out from
    the image of T, so dη(Q1)/dη(Q2) = s^i/(s^i + t) and the shed caustic
    lies at rho^d = s^i + t behind Q2; together
        sqrt(dη1/dη2) sqrt(rho^d/(s^d(rho^d + s^d))) = sqrt(s^i / (s^d (s^i + t + s^d))).
    The path is kept only if Q1 and Q2 lie on the lateral surface.
    """
    cx, cy, z0, hgt, a = cyl
    p = plan if plan is not None else cylinder_plan(T, cyl, R)
    dphi = p["dphi_plus"] if side > 0 else TWO_PI - p["dphi_plus"]
    phi = dphi - p["gT"] - p["gR"] + TWO_PI * ell
    dT, dR = p["dT"], p["dR"]
    L2 = dT + a * phi + dR
    dz = R[:, 2] - T[2]
    Stot = np.hypot(L2, dz)
    cosd = L2 / Stot
    sind = dz / Stot
    sI = dT / cosd
    t = a * phi / cosd
    sD = dR / cosd
    zQ1 = T[2] + dz * dT / L2
    zQ2 = T[2] + dz * (dT + a * phi) / L2
    alpha1 = p["aT"] + side * p["gT"]
    alpha2 = alpha1 + side * phi
    n1 = np.stack([np.cos(alpha1) * np.ones_like(phi), np.sin(alpha1) * np.ones_like(phi), np.zeros_like(phi)], 1)
    n2 = np.stack([np.cos(alpha2), np.sin(alpha2), np.zeros_like(phi)], 1)

    def tangent(nv):
        c = side * np.stack([-nv[:, 1], nv[:, 0], np.zeros_like(phi)], 1)
        return cosd[:, None] * c + sind[:, None] * np.array([0.0, 0.0, 1.0])

    t1 = tangent(n1)
    t2 = tangent(n2)
    b1 = np.cross(t1, n1)
    b2 = np.cross(t2, n2)
    base = np.array([cx, cy, 0.0])
    Q1 = base + a * n1
    Q1[:, 2] = zQ1
    Q2 = base + a * n2
    Q2[:, 2] = zQ2
    on_body = (zQ1 >= z0) & (zQ1 <= z0 + hgt) & (zQ2 >= z0) & (zQ2 <= z0 + hgt)
    ok = (p["rhoT"] > a) & (p["rhoR"] > a)
    S = np.sqrt(sI / (sD * (sI + t + sD))).astype(complex)
    return dict(kind="creep", valid=(phi >= 0) & on_body & ok, phi=phi, Q1=Q1, Q2=Q2,
                n1=n1, b1=b1, n2=n2, b2=b2, t1=t1, t2=t2, s_i=sI, t=t, s_d=sD,
                rho_g=a / cosd ** 2, S=S, rho_perp=np.full(phi.shape, np.inf))


def cylinder_reflection(T, cyl, R, plan=None):
    """Specular reflection on a vertical cylinder for lit receivers.

    Minimising the 3-D length over the reflection height at fixed azimuth
    splits dz in proportion to the projected lengths, so the azimuth solves the
    2-D Alhazen problem in projection (bisection on the arc seen from both
    T and R) and z_Q = T_z + dz |T'Q'| / (|T'Q'| + |Q'R'|).
    The surface curvature is (1/a) c c with c the circumferential unit vector;
    projecting it on the wavefront (Deschamps' phase matching) gives
        1/rho_1 = 1/s^i + 2 cos^2(beta)/(a cos th_i),  1/rho_2 = 1/s^i,
    beta the elevation of the incident ray, and the radius of curvature in the
    plane of incidence rho_g = a/cos^2(delta_R), delta_R the angle between
    the incidence plane's trace and c.
    """
    cx, cy, z0, hgt, a = cyl
    p = plan if plan is not None else cylinder_plan(T, cyl, R)
    phi_p = p["dphi_plus"] - p["gT"] - p["gR"]
    phi_m = (TWO_PI - p["dphi_plus"]) - p["gT"] - p["gR"]
    ok = (p["rhoT"] > a) & (p["rhoR"] > a)
    lit = ((phi_p < 0) | (phi_m < 0)) & ok
    Tp = np.array([T[0] - cx, T[1] - cy])
    Rp = np.stack([R[:, 0] - cx, R[:, 1] - cy], axis=1)
    # arc seen from both points, as an increasing interval of azimuth
    lo_p = p["aT"] + p["dphi_plus"] - p["gR"]
    hi_p = p["aT"] + p["gT"]
    lo_m = p["aT"] - p["gT"]
    hi_m = p["aT"] - (TWO_PI - p["dphi_plus"]) + p["gR"]
    use_p = phi_p < 0
    lo = np.where(use_p, lo_p, lo_m)
    hi = np.where(use_p, hi_p, hi_m)
    lo = np.where(lit, lo, 0.0)
    hi = np.where(lit, hi, 1.0)

    def g(al):
        qx, qy = a * np.cos(al), a * np.sin(al)
        tx, ty = -np.sin(al), np.cos(al)
        dt = np.hypot(qx - Tp[0], qy - Tp[1])
        dr = np.hypot(qx - Rp[:, 0], qy - Rp[:, 1])
        return ((qx - Tp[0]) * tx + (qy - Tp[1]) * ty) / dt + ((qx - Rp[:, 0]) * tx + (qy - Rp[:, 1]) * ty) / dr

    al = _bisect_stationary(g, lo, hi)
    qx, qy = a * np.cos(al), a * np.sin(al)
    lt = np.hypot(qx - Tp[0], qy - Tp[1])
    lr = np.hypot(qx - Rp[:, 0], qy - Rp[:, 1])
    dz = R[:, 2] - T[2]
    zQ = T[2] + dz * lt / (lt + lr)
    Q = np.stack([cx + qx, cy + qy, zQ], 1)
    n = np.stack([np.cos(al), np.sin(al), np.zeros_like(al)], 1)
    on_body = (zQ >= z0) & (zQ <= z0 + hgt)
    si_hat = _unit(Q - T)
    circ = np.stack([-np.sin(al), np.cos(al), np.zeros_like(al)], 1)
    tang = si_hat - np.einsum("ij,ij->i", si_hat, n)[:, None] * n
    tn2 = np.einsum("ij,ij->i", tang, tang)
    tc = np.einsum("ij,ij->i", tang, circ)
    cos2_dR = np.where(tn2 > 0, tc * tc / np.where(tn2 > 0, tn2, 1.0), 1.0)
    rho_g = a / np.maximum(cos2_dR, 1e-300)
    cos2_beta = 1.0 - si_hat[:, 2] ** 2
    out = _reflection_common(T, R, Q, n, lit & on_body, rho_g=rho_g,
                             inv_f1_cos=2.0 * cos2_beta / a,
                             inv_f2_over_cos=np.zeros_like(al))
    return out

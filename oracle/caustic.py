"""Uniform field of a sphere's creeping-ray pairs at the axial caustic, FP64
oracle.  Test infrastructure (see ``oracle/__init__``).

Every creeping ray of a sphere lies in a half-plane bounded by the source
axis (the line through the source T and the centre C).  A receiver R at
polar angle theta_R from e_T = (T - C)/|T - C| sees its rays in pairs that
meet on the axis: near the rear axis (theta_R -> pi) the paths (side +, ell)
and (side -, ell); near the front axis (theta_R -> 0) the paths
(side -, ell - 1) and (side +, ell).  The shorter one ("near") runs in R's
own half-plane, the longer one ("far") in the opposite half-plane and
crosses the axis before R.  Both ray fields grow as 1/sqrt(rho_perp) at the
axis (Eq. (4)'s divergence factor; the record's S).

The pair is the stationary-phase value of an integral over the azimuth
alpha of the half-plane a ray travels in (alpha = 0: the near ray's,
alpha = pi: the far ray's).  Near the axis its phase is k s_bar - x cos
alpha, with

    x = k (s_far - s_near)/2 = k a eps,  eps = pi - theta_R (rear) or theta_R (front),
    s_bar = (s_near + s_far)/2,

and the polarisation dyadic turns with alpha exactly: with u = e_T, e1 the
near ray's half-plane direction and e2 = u x e1, the half-plane at alpha has
rho(alpha) = cos(alpha) e1 + sin(alpha) e2, normals n1 = c1 u + s1 rho at Q1
and n2 = c2 u + s2 rho at Q2, and binormal b = -u x rho.  The scalar
amplitude of each polarisation is taken linear in cos(alpha) between its
values at the two rays, G(alpha) = G_bar + dG cos(alpha) with
G_bar = (G_near + G_far)/2, dG = (G_near - G_far)/2; for the hard part the
two components of n2 are interpolated apiece (H_u = G_h c2, H_rho = G_h s2),
so that each ray keeps its own Q2.  The integral is then closed with

    int_0^{2 pi} cos(n alpha) e^{j x cos alpha} d alpha = 2 pi j^n J_n(x).

Each G is the ray's amplitude with the transverse factor exchanged for its
finite limit,

    G = T_p |S| sqrt(x/(2 pi)) e^{j pi/4} e^{j pi n_s/2} e^{-j k s_bar} / s^i,
    |S| sqrt(x) = sqrt(a sin(gamma_T) k a eps / (s^d d_R sin eps)),

with T_p the ray's Fock transfer function of Eq. (4) and n_s the near
ray's caustic count, floor(theta2_near/pi).  The far ray has exactly one
caustic more (where it crosses the axis: in space, or on the surface at a
pole when its Q2 lies beyond one), and that quarter turn is what the Bessel
functions supply.  For large x, J_n's leading asymptotic form turns
the result back into the two ray fields of Eq. (4) exactly; on the axis it
is finite and independent of the direction from which the axis is reached.

Receivers with theta_R > pi/2 pair the paths at the rear axis, the others at
the front axis (where x is largest, so the switch moves the field by
O(1/x)).  A pair is evaluated this way only when both of its paths are valid
and visible; otherwise each ray keeps its own field.
"""
import numpy as np
from scipy.special import jv

from . import fock, geometry


def pair_keys(l_enc, rear):
    """(near, far) path keys (side, ell) of the pairs at the rear or the front axis."""
    if rear:
        return [((+1, l), (-1, l)) for l in range(l_enc + 1)]
    return [((-1, l - 1), (+1, l)) for l in range(1, l_enc + 1)]


def rear_mask(T, C, R):
    """True where the receiver pairs its paths at the rear axis (theta_R > pi/2)."""
    _, _, _, _, thR = geometry.sphere_frame(T, C, 0.0, R)
    return thR > 0.5 * np.pi


def _transfer(rec, idx, k, hard):
    """The ray's Fock transfer function T_p of Eq. (4), as the field assembly forms it."""
    rho_g = rec["rho_g"][idx]
    sI, t, sD = rec["s_i"][idx], rec["t"][idx], rec["s_d"][idx]
    m = (k * rho_g / 2) ** (1.0 / 3.0)
    xi = m * t / rho_g
    L = sI * sD / (sI + sD)
    X = k * L * xi ** 2 / (2 * m * m)
    q = np.sqrt(k * L / 2) / m
    return -m * np.sqrt(2 / k) * fock.shadow_B(xi, X, q, hard)


def add_pair(acc, T, C, a, R, near, far, idx, rear, dip, amp, k, mode):
    """Adds the uniform field of the pair (near, far) at receivers idx into
    acc (acc[idx] for mode 'soft'/'hard', acc[:, idx] for 'em')."""
    Ri = R[idx]
    dT, u, dR, eperp, thR = geometry.sphere_frame(T, C, a, Ri)
    eps = np.pi - thR if rear else thR
    x = k * a * eps
    sI = np.sqrt(dT * dT - a * a)
    sD = np.sqrt(dR * dR - a * a)
    gT = np.arctan2(sI, a)
    c1, s1 = np.cos(gT), np.sin(gT)
    # near ray's half-plane: side + runs in R's own (eperp), side - in the other
    e1 = eperp if rear else -eperp
    # close to the axis the rounding of R - C leaves e1 a component along u
    # of order 1e-16 |R - C| / rho_perp; removed, so that p1 e1 + p2 e2 is
    # the transverse dipole whatever the direction of e1
    e1 = e1 - (e1 @ u)[:, None] * u[None, :]
    e1 = e1 / np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(np.broadcast_to(u, e1.shape), e1)
    ratio = np.where(eps > 0, eps / np.where(eps > 0, np.sin(eps), 1.0), 1.0)
    s_x = np.sqrt(a * s1 * k * a * ratio / (sD * dR))          # |S| sqrt(x)
    s_n = near["s_i"][idx] + near["t"][idx] + near["s_d"][idx]
    s_f = far["s_i"][idx] + far["t"][idx] + far["s_d"][idx]
    s_bar = 0.5 * (s_n + s_f)
    base = s_x / np.sqrt(2 * np.pi) * np.exp(0.25j * np.pi) * np.exp(-1j * k * s_bar) / sI
    th2 = [gT + rec["phi"][idx] for rec in (near, far)]
    sn = np.exp(0.5j * np.pi * np.floor(th2[0] / np.pi))
    surf = [sn, sn]
    J = [jv(n, x) for n in range(4)]
    A0 = 2 * np.pi * J[0]
    A1 = 2j * np.pi * J[1]
    Am = np.pi * (J[0] - J[2])
    Ap = np.pi * (J[0] + J[2])
    B3 = 0.5j * np.pi * (3 * J[1] - J[3])
    B1 = 0.5j * np.pi * (J[1] + J[3])
    if mode in ("soft", "hard"):
        G = [_transfer(rec, idx, k, mode == "hard") * base * sf for rec, sf in zip((near, far), surf)]
        Gb, dG = 0.5 * (G[0] + G[1]), 0.5 * (G[0] - G[1])
        acc[idx] += Gb * A0 + dG * A1
        return
    Gs = [_transfer(rec, idx, k, False) * base * sf for rec, sf in zip((near, far), surf)]
    Gh = [_transfer(rec, idx, k, True) * base * sf for rec, sf in zip((near, far), surf)]
    Hu = [g * np.cos(t2) for g, t2 in zip(Gh, th2)]
    Hr = [g * np.sin(t2) for g, t2 in zip(Gh, th2)]
    # the far ray's Q2 sits in the half-plane -e1: its n2 = c2 u + s2 (-e1),
    # which is the interpolation's value at alpha = pi
    mean = lambda v: 0.5 * (v[0] + v[1])
    half = lambda v: 0.5 * (v[0] - v[1])
    Gsb, dGs, Hub, dHu, Hrb, dHr = mean(Gs), half(Gs), mean(Hu), half(Hu), mean(Hr), half(Hr)
    p = np.asarray(dip, dtype=float)
    pu = float(p @ u)
    p1 = e1 @ p
    p2 = e2 @ p
    Es_1 = p1 * (Gsb * Ap + dGs * B1)
    Es_2 = p2 * (Gsb * Am + dGs * B3)
    Eh_u = c1 * pu * (Hub * A0 + dHu * A1) + s1 * p1 * (Hub * A1 + dHu * Am)
    Eh_1 = c1 * pu * (Hrb * A1 + dHr * Am) + s1 * p1 * (Hrb * Am + dHr * B3)
    Eh_2 = s1 * p2 * (Hrb * Ap + dHr * B1)
    E = amp * (Eh_u[:, None] * u[None, :] + (Es_1 + Eh_1)[:, None] * e1 + (Es_2 + Eh_2)[:, None] * e2)
    acc[:, idx] += E.T

"""Two-dimensional UTD field of a line source beside a PEC circular cylinder.

Test infrastructure (see ``oracle/__init__``).  This is the oracle's cylinder
geometry and Fock machinery with the spreading of a cylindrical wave: the
source is a line parallel to the axis, the incident ray field is
u^i = e^{-jks}/sqrt(s), the creeping field has no transverse spreading
(dη ratio 1, rho^d = inf) and the reflected field keeps only the in-plane
caustic, 1/rho_1 = 1/s^i + 2/(a cos th_i).  It exists to compare the oracle's
cylinder formulas against the exact Hankel series in ``mie``.
"""
import numpy as np

from . import fock, geometry

C0 = 299792458.0


def field2d(cyl_xy_a, src_xy, rx_xy, f, hard=False, l_enc=0):
    cx, cy, a = cyl_xy_a
    k = 2 * np.pi * f / C0
    T = np.array([src_xy[0], src_xy[1], 0.0])
    R = np.column_stack([rx_xy, np.zeros(len(rx_xy))])
    cyl = (cx, cy, -1e9, 2e9, a)
    plan = geometry.cylinder_plan(T, cyl, R)
    u = np.zeros(R.shape[0], dtype=complex)
    # line of sight: the receiver is lit on exactly one side or the segment misses the disc
    lit = np.zeros(R.shape[0], dtype=bool)
    for side in (+1, -1):
        dphi = plan["dphi_plus"] if side > 0 else 2 * np.pi - plan["dphi_plus"]
        lit |= dphi - plan["gT"] - plan["gR"] < 0
    s = np.hypot(R[:, 0] - T[0], R[:, 1] - T[1])
    u[lit] += np.exp(-1j * k * s[lit]) / np.sqrt(s[lit])
    for side in (+1, -1):
        for ell in range(l_enc + 1):
            rec = geometry.cylinder_creeping(T, cyl, R, side, ell, plan)
            v = rec["valid"]
            sI, t, sD = rec["s_i"][v], rec["t"][v], rec["s_d"][v]
            m = (k * a / 2) ** (1 / 3)
            xi = m * t / a
            L = sI * sD / (sI + sD)
            X = k * L * xi ** 2 / (2 * m * m)
            q = np.sqrt(k * L / 2) / m
            Tp = -m * np.sqrt(2 / k) * fock.shadow_B(xi, X, q, hard)
            u[v] += Tp * np.exp(-1j * k * (sI + t + sD)) / np.sqrt(sI) / np.sqrt(sD)
    rec = geometry.cylinder_reflection(T, cyl, R, plan)
    v = rec["valid"]
    if v.any():
        sI, sR, ci = rec["s_i"][v], rec["s_r"][v], rec["cos_i"][v]
        m = (k * a / 2) ** (1 / 3)
        xi = -2 * m * ci
        L = sI * sR / (sI + sR)
        X = 2 * k * L * ci ** 2
        q = np.sqrt(k * L / 2) / m
        rho1_over_cos = 1.0 / (ci / sI + 2.0 / a)
        rho1 = rho1_over_cos * ci
        Rb = fock.lit_Rbar(xi, X, q, hard)
        spread = 2 * np.sqrt(rho1_over_cos / (2 * m)) / np.sqrt(rho1 + sR)
        u[v] += Rb * spread * np.exp(-1j * k * (sI + sR)) / np.sqrt(sI)
    return u


def exact_normalisation(f):
    """H_0^{(2)}(ks) ~ sqrt(2/(pi k)) e^{j pi/4} e^{-jks}/sqrt(s)."""
    k = 2 * np.pi * f / C0
    return np.sqrt(2 / (np.pi * k)) * np.exp(1j * np.pi / 4)

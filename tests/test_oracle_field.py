"""Pins of the oracle's field assembly: exact series, reciprocity, continuity
across the shadow boundary, the flat-plate limit, brute-force geometry and
occlusion."""
import numpy as np
import pytest

from oracle import cyl2d, field, geometry, mie, occlusion

C0 = 299792458.0


def _ring(n, r=3.0, upper=False):
    ph = (np.pi if upper else 2 * np.pi) * (np.arange(n) + 0.5) / n
    return ph, np.stack([r * np.cos(ph), r * np.sin(ph), np.zeros(n)], 1)


# ---------------------------------------------------------------------------
# exact solutions
# ---------------------------------------------------------------------------

def test_series_conventions_match_closed_forms():
    """The expansions used by the exact solutions reproduce the free-space
    fields they expand (scalar Green's function; curl curl of a dipole)."""
    k = 2 * np.pi * 1e9 / C0
    b = 3.0
    r = np.array([2.0, 2.5, 3.6, 4.0])
    th = np.array([0.4, 1.3, 2.0, 2.9])
    s = mie.sphere_scalar_incident_series(k, b, r, th, 150)
    R = np.sqrt(r * r + b * b - 2 * r * b * np.cos(th))
    np.testing.assert_allclose(s, np.exp(-1j * k * R) / R, rtol=1e-9)
    Er, Et = mie.radial_dipole_debye(k, b, r, th, 150, "incident")
    P = np.stack([r * np.sin(th), 0 * r, r * np.cos(th)], 1)
    E = mie.dipole_free_field(np.array([0, 0, b]), np.array([0, 0, 1.0]), P, k)
    rh = np.stack([np.sin(th), 0 * r, np.cos(th)], 1)
    thh = np.stack([np.cos(th), 0 * r, -np.sin(th)], 1)
    np.testing.assert_allclose(Er, np.einsum("ij,ij->i", E, rh), rtol=1e-8)
    np.testing.assert_allclose(Et, np.einsum("ij,ij->i", E, thh), rtol=1e-8)


@pytest.mark.parametrize("mode,max_db,rms_db,lit_db", [("soft", 1.9, 0.6, 0.05), ("hard", 1.5, 0.35, 0.35)])
def test_scalar_sphere_vs_mie(mode, max_db, rms_db, lit_db):
    """Sphere-ring geometry (a = 0.5 m, source at 3 m, ring r = 3 m, 1 GHz,
    ka = 10.5) against the exact series.  The leading-order UTD neglects
    O(m^-2) ~ 0.33 terms at m = 1.74; excluded: within 10 deg of the source
    and within 3 deg of the axial caustic."""
    f, a = 1e9, 0.5
    k = 2 * np.pi * f / C0
    ph, rx = _ring(4096)
    u = field.field(dict(spheres=[[0, 0, 0, a]]), dict(pos=[3.0, 0, 0]), rx, [f], mode=mode)[0]
    th = np.arccos(np.clip(np.cos(ph), -1, 1))
    ue = mie.sphere_scalar(k, a, 3.0, np.full(ph.size, 3.0), th, hard=(mode == "hard"))
    dB = 20 * np.log10(np.abs(u) / np.abs(ue))
    deg = np.degrees(th)
    sel = (deg > 10) & (deg < 177)
    assert np.max(np.abs(dB[sel])) < max_db
    assert np.sqrt(np.mean(dB[sel] ** 2)) < rms_db
    lit = (deg > 10) & (deg < 140)
    assert np.max(np.abs(dB[lit])) < lit_db        # GO + Fock reflection region


def test_em_radial_dipole_vs_mie_improves_with_ka():
    """Radial electric dipole (hard polarisation) against the exact Debye
    series: within 0.2 dB in the lit region, and the shadow error falls with
    ka as the neglected O(m^-2) terms do."""
    a, b = 0.5, 3.0
    ph, rx = _ring(1024, upper=True)
    deg = np.degrees(ph)
    worst = []
    for f in (1e9, 3e9, 6e9):
        k = 2 * np.pi * f / C0
        E = field.field(dict(spheres=[[0, 0, 0, a]]), dict(pos=[b, 0, 0], dipole=[1.0, 0, 0]), rx, [f])[0]
        Mr, Mt = mie.sphere_radial_dipole(k, a, b, np.stack([np.full(ph.size, 3.0), ph], 1))
        mag_u = np.linalg.norm(np.abs(E), axis=0)
        mag_m = np.sqrt(np.abs(Mr) ** 2 + np.abs(Mt) ** 2) / k ** 2
        dB = 20 * np.log10(mag_u / mag_m)
        assert np.max(np.abs(dB[(deg > 10) & (deg < 120)])) < 0.2
        worst.append(np.max(np.abs(dB[(deg > 150) & (deg < 172)])))
    # neglected terms scale as m^-2 = (ka/2)^(-2/3): ratios 3^(2/3), 2^(2/3)
    assert worst[0] < 4.5 and worst[2] < 1.6
    np.testing.assert_allclose([worst[0] / worst[1], worst[1] / worst[2]], [3 ** (2 / 3), 2 ** (2 / 3)], rtol=0.3)


@pytest.mark.parametrize("hard", [False, True])
def test_cylinder_2d_vs_hankel_series(hard):
    """Line source beside a PEC cylinder: the oracle's cylinder geometry and
    Fock functions against the exact eigenfunction series (ka = 10.5)."""
    f, a = 1e9, 0.5
    k = 2 * np.pi * f / C0
    ph = np.pi * (np.arange(512) + 0.5) / 512
    rx = np.stack([3 * np.cos(ph), 3 * np.sin(ph)], 1)
    u = cyl2d.field2d((0, 0, a), (3.0, 0), rx, f, hard)
    ue = mie.cylinder_line_source(k, a, 3.0, np.full(ph.size, 3.0), ph, hard) / cyl2d.exact_normalisation(f)
    dB = 20 * np.log10(np.abs(u) / np.abs(ue))
    sel = (np.degrees(ph) > 10) & (np.degrees(ph) < 178)
    assert np.max(np.abs(dB[sel])) < 0.4


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_reciprocity_many_bodies():
    """q . E_p(R) = p . E_q(T) for dipoles p at T and q at R, with spheres and
    finite cylinders occluding each other."""
    rng = np.random.default_rng(5)
    scene = dict(spheres=[[0, 0, 0, 0.7], [2.5, 1.0, 0.3, 0.4]],
                 cylinders=[[-1.5, 2.0, -1.0, 3.0, 0.3], [1.0, -2.5, -2.0, 2.5, 0.25]])
    for _ in range(6):
        T = rng.uniform(-4, 4, 3)
        R = rng.uniform(-4, 4, (1, 3))
        p, q = rng.normal(size=3), rng.normal(size=3)
        if field.source_inside(scene, T) or field.source_inside(scene, R[0]):
            continue
        Ep = field.field(scene, dict(pos=T, dipole=p), R, [2.4e9, 5e9], opts=dict(l_enc=1))[:, :, 0]
        Eq = field.field(scene, dict(pos=R[0], dipole=q), T[None, :], [2.4e9, 5e9], opts=dict(l_enc=1))[:, :, 0]
        a, b = Ep @ q, Eq @ p
        assert np.max(np.abs(a - b) / np.abs(a)) < 1e-11


@pytest.mark.parametrize("body", ["sphere", "cylinder"])
def test_shadow_boundary_continuity(body):
    """The total field is continuous across the shadow boundary (the paper's
    claim for smooth-surface UTD, Sec. III-B): the jump shrinks linearly with
    the distance from the boundary."""
    f = 3e9
    if body == "sphere":
        a, T, d = 1.0, np.array([4.0, 0, 0]), 5.0
        scene = dict(spheres=[[0, 0, 0, a]])
        z = 0.0
    else:
        a, T, d = 0.5, np.array([3.0, 0, 1.0]), 4.0
        scene = dict(cylinders=[[0, 0, -5, 10, a]])
        z = -0.7
    thb = np.arccos(a / np.hypot(T[0], T[1])) + np.arccos(a / d)
    jumps = []
    for dth in (1e-4, 1e-6):
        th = np.array([thb - dth, thb + dth])
        rx = np.stack([d * np.cos(th), d * np.sin(th), np.full(2, z)], 1)
        for dip in ([0, 0, 1.0], [1.0, 0, 0], [0.3, 0.5, 0.8]):
            E = field.field(scene, dict(pos=T, dipole=dip), rx, [f])[0]
            jumps.append(np.max(np.abs(E[:, 0] - E[:, 1])) / np.max(np.abs(E[:, 0])))
    jumps = np.array(jumps).reshape(2, 3)
    assert np.all(jumps[1] < 2e-3)
    np.testing.assert_allclose(jumps[1] / jumps[0], 1e-2, rtol=0.05)


def test_flat_plate_limit_is_image_dipole():
    """A sphere of radius 1e6 m looks like a PEC plane near its top: the
    reflected field tends to that of the image dipole (the sag of the surface
    over 2 m shifts the path by ~1e-6 m, i.e. 1e-4 rad)."""
    A = 1e6
    scene = dict(spheres=[[0, 0, -A, A]])
    T = np.array([0.0, 0.0, 1.0])
    rx = np.array([[3.0, 0.5, 2.0], [1.0, -2.0, 0.5], [-2.5, 1.5, 1.2]])
    f = 2.4e9
    k = 2 * np.pi * f / C0
    p = np.array([0.4, -0.3, 0.8])
    E, info = field.field(scene, dict(pos=T, dipole=p), rx, [f], return_info=True)
    los = E[0] - field.field(scene, dict(pos=T, dipole=p), rx, [f], opts=dict(lit_branch=True),
                             frozen=_only_los(info))[0]
    img = np.array([0.0, 0.0, -1.0])
    pim = np.array([-p[0], -p[1], p[2]])
    v = rx - img
    s = np.linalg.norm(v, axis=1)
    sh = v / s[:, None]
    Eimg = (pim[None, :] - (sh @ pim)[:, None] * sh) * (np.exp(-1j * k * s) / s)[:, None]
    assert np.max(np.abs(los.T - Eimg)) / np.max(np.abs(Eimg)) < 1e-3


def _only_los(info):
    fr = dict(los=info["los"], inside=info["inside"], flags=info["flags"], paths=[])
    for key, rec in info["paths"]:
        r = dict(rec)
        r["valid"] = np.zeros_like(rec["valid"])
        fr["paths"].append((key, r))
    return fr


def test_frozen_classification_reproduces_field():
    scene = dict(spheres=[[0, 0, 0, 0.7]], cylinders=[[-1.5, 2.0, -1.0, 3.0, 0.3]])
    tx = dict(pos=[3.0, 0.5, 0.2], dipole=[0.2, 0.3, 0.9])
    rng = np.random.default_rng(2)
    rx = rng.uniform(-4, 4, (64, 3))
    E, info = field.field(scene, tx, rx, [3e9], return_info=True)
    E2 = field.field(scene, tx, rx, [3e9], frozen=info)
    np.testing.assert_array_equal(E, E2)


def test_receiver_inside_body_is_zero_and_flagged():
    scene = dict(spheres=[[0, 0, 0, 1.0]], cylinders=[[3, 3, 0, 2, 0.5]])
    rx = np.array([[0.2, 0.1, 0.0], [3.1, 3.0, 1.0], [3.1, 3.0, 2.5], [-3, 0, 0]])
    E, info = field.field(scene, dict(pos=[5.0, 0, 0.5]), rx, [1e9], return_info=True)
    assert np.all(E[0, :, :2] == 0)
    assert np.all(info["flags"][:2] & field.FLAG_INSIDE)
    assert not np.any(info["flags"][2:] & field.FLAG_INSIDE)
    assert np.all(np.abs(E[0, :, 2:]) .sum(axis=0) > 0)


def test_encircling_paths_are_small_but_present():
    """Lit receivers also get the long-way creeping wave (interference in the
    lit region, Sec. III-B); an extra encirclement is exponentially weaker."""
    ph, rx = _ring(64)
    sc = dict(spheres=[[0, 0, 0, 0.5]])
    tx = dict(pos=[3.0, 0, 0], dipole=[1.0, 0, 0])
    E0 = field.field(sc, tx, rx, [1e9])
    E1 = field.field(sc, tx, rx, [1e9], opts=dict(l_enc=1))
    d = np.linalg.norm(E1 - E0, axis=1)[0]
    assert np.all(d > 0) and np.max(d / np.linalg.norm(E0, axis=1)[0]) < 2e-3


# ---------------------------------------------------------------------------
# geometry against brute force
# ---------------------------------------------------------------------------

def test_sphere_creeping_is_shortest_wrapped_path():
    """Total length s^i + t + s^d is the minimum over all wrapped paths
    T -> Q1 -> (great-circle arc) -> Q2 -> R in the T-C-R plane; and R lies
    on the tangent ray shed from Q2."""
    T = np.array([2.5, 0.3, 0.4])
    R = np.array([[-2.0, 0.8, -0.5]])
    a = 0.8
    rec = geometry.sphere_creeping(T, np.zeros(3), a, R, +1, 0)
    L = rec["s_i"][0] + rec["t"][0] + rec["s_d"][0]
    np.testing.assert_allclose(rec["Q2"][0] + rec["s_d"][0] * rec["t2"][0], R[0], atol=1e-12)
    np.testing.assert_allclose(np.dot(rec["Q1"][0] - T, rec["n1"][0]), 0, atol=1e-12)
    dT, eT, dR, ep, thR = geometry.sphere_frame(T, np.zeros(3), a, R)
    th = np.linspace(0, np.pi, 2001)
    T2 = np.array([dT, 0.0])
    R2 = np.array([dR[0] * np.cos(thR[0]), dR[0] * np.sin(thR[0])])
    best = np.inf
    for t1 in th[th <= np.arccos(a / dT)]:
        for t2 in th[(th >= t1) & (th >= thR[0] - np.arccos(a / dR[0]))][::5]:
            q1 = a * np.array([np.cos(t1), np.sin(t1)])
            q2 = a * np.array([np.cos(t2), np.sin(t2)])
            best = min(best, np.linalg.norm(q1 - T2) + a * (t2 - t1) + np.linalg.norm(R2 - q2))
    assert L <= best + 1e-12 and best - L < 2e-5


def test_cylinder_helix_is_shortest_path():
    """The helical path against a direct minimisation of
    |T - Q1| + geodesic(Q1, Q2) + |Q2 - R| over the attachment points."""
    from scipy.optimize import minimize
    cyl = (0.3, -0.2, -2.0, 5.0, 0.4)
    T = np.array([2.0, 0.5, 1.5])
    R = np.array([[-1.8, -0.9, -0.6]])
    rec = geometry.cylinder_creeping(T, cyl, R, +1, 0)
    assert rec["valid"][0]
    L = rec["s_i"][0] + rec["t"][0] + rec["s_d"][0]
    cx, cy, z0, h, a = cyl
    a1 = np.arctan2(rec["Q1"][0, 1] - cy, rec["Q1"][0, 0] - cx)
    a2 = np.arctan2(rec["Q2"][0, 1] - cy, rec["Q2"][0, 0] - cx)
    if a2 < a1:
        a2 += 2 * np.pi

    def length(x):
        al1, z1, al2, z2 = x
        q1 = np.array([cx + a * np.cos(al1), cy + a * np.sin(al1), z1])
        q2 = np.array([cx + a * np.cos(al2), cy + a * np.sin(al2), z2])
        return np.linalg.norm(q1 - T) + np.hypot(a * (al2 - al1), z2 - z1) + np.linalg.norm(R[0] - q2)

    def visible(x):
        # Q1 seen from T and Q2 seen from R: the straight legs stay outside
        al1, z1, al2, z2 = x
        n1 = np.array([np.cos(al1), np.sin(al1)])
        n2 = np.array([np.cos(al2), np.sin(al2)])
        return [n1 @ (T[:2] - np.array([cx, cy])) - a, n2 @ (R[0, :2] - np.array([cx, cy])) - a]

    x0 = np.array([a1 - 0.05, rec["Q1"][0, 2] + 0.1, a2 + 0.05, rec["Q2"][0, 2] - 0.1])
    res = minimize(length, x0, method="SLSQP", constraints=[dict(type="ineq", fun=visible)],
                   options=dict(ftol=1e-15, maxiter=2000))
    assert abs(res.fun - L) < 1e-8
    np.testing.assert_allclose([res.x[1], res.x[3]], [rec["Q1"][0, 2], rec["Q2"][0, 2]], atol=1e-4)


@pytest.mark.parametrize("body", ["sphere", "cylinder"])
def test_reflection_point_minimises_path(body):
    rng = np.random.default_rng(7)
    if body == "sphere":
        T = np.array([3.0, 0.4, 0.2])
        R = rng.uniform(-1, 1, (20, 3)) + np.array([2.5, 1.5, 0.0])
        rec = geometry.sphere_reflection(T, np.zeros(3), 0.9, R)
    else:
        cyl = (0.0, 0.0, -3.0, 6.0, 0.6)
        T = np.array([3.0, 0.4, 1.2])
        R = rng.uniform(-1, 1, (20, 3)) + np.array([2.5, 1.5, 0.0])
        rec = geometry.cylinder_reflection(T, cyl, R)
    ok = rec["valid"]
    assert ok.sum() > 10
    Q = rec["Q"][ok]
    n = rec["n"][ok]
    L0 = np.linalg.norm(Q - T, axis=1) + np.linalg.norm(R[ok] - Q, axis=1)
    # equal angles: reflected direction is the mirror of the incident one
    si = rec["si_hat"][ok]
    sr = rec["sr_hat"][ok]
    mirror = si - 2 * np.einsum("ij,ij->i", si, n)[:, None] * n
    np.testing.assert_allclose(sr, mirror, atol=1e-9)
    # brute force: no nearby surface point gives a shorter path
    for i in range(Q.shape[0]):
        for dv in rng.normal(size=(50, 3)) * 1e-3:
            if body == "sphere":
                q = Q[i] + dv
                q = q / np.linalg.norm(q) * 0.9
            else:
                q = Q[i] + dv
                r = np.hypot(q[0], q[1])
                q[:2] *= 0.6 / r
            assert np.linalg.norm(q - T) + np.linalg.norm(R[ok][i] - q) >= L0[i] - 1e-12


def _reflect_ray(T, d, body):
    """Exact reflection of the ray T + s d on a sphere (C, a) or infinite
    vertical cylinder (cx, cy, a): hit point and reflected direction."""
    if body[0] == "s":
        C, a = body[1], body[2]
        w = T - C
        b = d @ w
        c = w @ w - a * a
        s = -b - np.sqrt(b * b - c)
        P = T + s * d
        n = (P - C) / a
    else:
        cx, cy, a = body[1], body[2], body[3]
        wx, wy = T[0] - cx, T[1] - cy
        A = d[0] ** 2 + d[1] ** 2
        B = d[0] * wx + d[1] * wy
        Cc = wx * wx + wy * wy - a * a
        s = (-B - np.sqrt(B * B - A * Cc)) / A
        P = T + s * d
        n = np.array([P[0] - cx, P[1] - cy, 0.0]) / a
    r = d - 2 * (d @ n) * n
    return P, r


@pytest.mark.parametrize("body", ["sphere", "cylinder"])
def test_reflection_spreading_against_ray_tube(body):
    """sqrt(rho1 rho2 / ((rho1 + s)(rho2 + s))) against the area of a thin
    bundle of exactly reflected rays (finite-difference Jacobian)."""
    T = np.array([3.0, 0.4, 1.1])
    R = np.array([[2.2, 2.0, -0.3]])
    if body == "sphere":
        rec = geometry.sphere_reflection(T, np.zeros(3), 0.9, R)
        bd = ("s", np.zeros(3), 0.9)
    else:
        rec = geometry.cylinder_reflection(T, (0.0, 0.0, -3.0, 6.0, 0.6), R)
        bd = ("c", 0.0, 0.0, 0.6)
    assert rec["valid"][0]
    Q, sr = rec["Q"][0], rec["sr_hat"][0]
    d0 = (Q - T) / np.linalg.norm(Q - T)
    e1 = np.cross(d0, [0.3, 0.1, 0.9])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d0, e1)
    h = 1e-6

    def plane_hit(u, v, dist):
        d = d0 + u * e1 + v * e2
        d /= np.linalg.norm(d)
        P, r = _reflect_ray(T, d, bd)
        c = Q + dist * sr
        s = ((c - P) @ sr) / (r @ sr)
        return P + s * r

    areas = []
    for dist in (0.0, rec["s_r"][0]):
        pu = (plane_hit(h, 0, dist) - plane_hit(-h, 0, dist)) / (2 * h)
        pv = (plane_hit(0, h, dist) - plane_hit(0, -h, dist)) / (2 * h)
        areas.append(np.linalg.norm(np.cross(pu, pv)))
    df2 = areas[0] / areas[1]
    rho1, rho2, s = rec["rho1"][0], rec["rho2"][0], rec["s_r"][0]
    np.testing.assert_allclose(df2, rho1 * rho2 / ((rho1 + s) * (rho2 + s)), rtol=1e-5)


def _helix_length(T, cyl, P, side, ell):
    r = geometry.cylinder_creeping(T, cyl, np.atleast_2d(P), side, ell)
    return (r["s_i"] + r["t"] + r["s_d"])[0]


@pytest.mark.parametrize("R,side,ell", [((-2.5, 1.0, 0.3), -1, 0), ((-2.5, -1.2, 0.3), 1, 0),
                                        ((-1.0, -2.7, -0.5), 1, 1), ((0.4, 2.2, 3.3), -1, 0)])
def test_cylinder_creeping_spreading_against_wavefronts(R, side, ell):
    """The helical creeping spreading S^2 = (deta1/deta2) rho^d/(s^d (rho^d + s^d))
    (Eq. (4) on an obliquely illuminated cylinder) against the curvatures of
    the wavefronts of the path-length function psi = s^i + t + s^d, taken by
    finite differences (psi itself is pinned by the brute-force shortest
    path):
    * in space at R, the Hessian of psi across the shed ray has the
      eigenvalues 1/s^d (the caustic of the shed rays on the surface) and
      1/(s^d + rho^d) (the second caustic, rho^d behind Q2);
    * on the surface, psi's second derivative across the surface ray is
      1/D, D the distance to the virtual source of the surface-ray fan, and
      deta1/deta2 = D(Q1)/D(Q2).
    A dropped t (rho^d = s^i, or deta ratio 1) fails both."""
    T = np.array([3.0, 0.4, 2.1])
    cyl = (0.0, 0.0, -1.0, 5.0, 0.6)
    R = np.array(R)
    rec = geometry.cylinder_creeping(T, cyl, R[None, :], side, ell)
    assert rec["valid"][0] and abs(R[2] - T[2]) > 1.0
    sI, t, sD = rec["s_i"][0], rec["t"][0], rec["s_d"][0]
    h = 1e-4
    E = np.eye(3)
    f = lambda P: _helix_length(T, cyl, P, side, ell)
    g = np.array([(f(R + h * E[i]) - f(R - h * E[i])) / (2 * h) for i in range(3)])
    H = np.array([[(f(R + h * E[i] + h * E[j]) - f(R + h * E[i] - h * E[j]) - f(R - h * E[i] + h * E[j])
                    + f(R - h * E[i] - h * E[j])) / (4 * h * h) for j in range(3)] for i in range(3)])
    u = g / np.linalg.norm(g)
    Pj = np.eye(3) - np.outer(u, u)
    lam = np.sort(np.linalg.eigvalsh(Pj @ H @ Pj))[1:]
    np.testing.assert_allclose(lam[1], 1.0 / sD, rtol=1e-5)
    rho_fd = 1.0 / lam[0] - sD
    np.testing.assert_allclose(rho_fd, sI + t, rtol=1e-5)
    assert abs(rho_fd - sI) > 1e-2 * sI

    def surface_radius(Q, tv, l):
        # psi on the surface along the surface direction normal to the ray
        a = cyl[4]
        th = np.arctan2(Q[1] - cyl[1], Q[0] - cyl[0])
        circ = np.array([-np.sin(th), np.cos(th), 0.0])
        bc, bz = -tv[2], tv @ circ
        hh = 1e-3
        v = [_helix_length(T, cyl, np.array([cyl[0] + a * np.cos(th + k * hh * bc / a),
                                              cyl[1] + a * np.sin(th + k * hh * bc / a), Q[2] + k * hh * bz]),
                           side, l) for k in (-1, 0, 1)]
        return hh * hh / (v[0] - 2 * v[1] + v[2])

    D1 = surface_radius(rec["Q1"][0], rec["t1"][0], 0)      # the surface wave just after attachment
    D2 = surface_radius(rec["Q2"][0], rec["t2"][0], ell)
    np.testing.assert_allclose([D1, D2], [sI, sI + t], rtol=1e-6)
    S2_fd = (D1 / D2) * rho_fd / (sD * (rho_fd + sD))
    np.testing.assert_allclose(abs(rec["S"][0]) ** 2, S2_fd, rtol=1e-5)


# ---------------------------------------------------------------------------
# occlusion
# ---------------------------------------------------------------------------

def test_grid_occlusion_equals_brute_force():
    rng = np.random.default_rng(11)
    tri = rng.uniform(0, 4, (400, 1, 3)) + rng.normal(scale=0.3, size=(400, 3, 3))
    p0 = rng.uniform(-0.5, 4.5, (3000, 3))
    p1 = rng.uniform(-0.5, 4.5, (3000, 3))
    g = occlusion.segments_vs_triangles(tri, p0, p1)
    b = occlusion.segments_vs_triangles(tri, p0, p1, brute=True)
    np.testing.assert_array_equal(g, b)
    assert 0.2 < g.mean() < 0.95


def test_body_occlusion_against_sampling():
    rng = np.random.default_rng(12)
    p0 = rng.uniform(-2, 2, (4000, 3))
    p1 = rng.uniform(-2, 2, (4000, 3))
    sph = (0.1, -0.2, 0.3, 0.7)
    cyl = (-0.3, 0.4, -0.5, 1.2, 0.5)
    t = np.linspace(0, 1, 4001)[1:-1]
    pts = p0[:, None, :] + t[None, :, None] * (p1 - p0)[:, None, :]
    in_s = (np.sum((pts - np.array(sph[:3])) ** 2, axis=2) <= sph[3] ** 2).any(axis=1)
    in_c = (((pts[..., 0] - cyl[0]) ** 2 + (pts[..., 1] - cyl[1]) ** 2 <= cyl[4] ** 2)
            & (pts[..., 2] >= cyl[2]) & (pts[..., 2] <= cyl[2] + cyl[3])).any(axis=1)
    hs = occlusion.segments_vs_sphere(p0, p1, sph)
    hc = occlusion.segments_vs_cylinder(p0, p1, cyl)
    # sampling can only miss grazing chords
    assert np.all(hs[in_s]) and np.mean(hs != in_s) < 2e-3
    assert np.all(hc[in_c]) and np.mean(hc != in_c) < 2e-3

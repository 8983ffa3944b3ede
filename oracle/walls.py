"""Single specular wall bounces (GO multipath) and the body paths they feed,
FP64 oracle.

Test infrastructure (see ``oracle/__init__``).

The scene triangles act as reflectors as well as occluders.  A reflector is
one plane of the triangle soup: all triangles lying in the same plane (unit
normal n, offset d, n.x = d) reflect as one mirror, and a specular point Q
on that plane counts only when it lies on one of those triangles.  The wall
material is a homogeneous slab (relative permittivity eps_r, conductivity
sigma, thickness t; or a perfect conductor), whose plane-wave reflection
coefficients for the two polarisations are those of a lossy dielectric slab
with its multiple internal reflections summed.

For a planar mirror the reflected wave is exactly the wave of the image
source T' = T - 2 (n.T - d) n seen through the mirror, so the paths that
reach a receiver R through one wall bounce are (Fig. 1: an earlier
interaction point acts as an equivalent source for the surface-diffracted
path; Eqs. (1)-(4) otherwise unchanged):

  wall           T -> Q_w -> R                   the image source's direct ray
  wall, body     T -> Q_w -> body -> R           creeping paths and the body
                                                 reflection of Eqs. (3)-(4)
                                                 with T' as the source
  body, wall     T -> body -> Q_w -> R           the same with the receiver's
                                                 image R' = R - 2 (n.R - d) n

The wall reflection maps the incident polarisation (amplitude-weighted
vector v on the ray direction s_in) to R_perp (v.e_perp) e_perp +
R_par (v.e_par_in) e_par_out with e_perp = s_in x n / |.|,
e_par = e_perp x s, and keeps the ray tube's spreading, so every path length
and spreading factor is that of the image construction.  Each path is gated
by the visibility of all its legs (the legs that end on a body do not test
that body; the open-segment rule leaves the legs' end points on the wall).
"""
import numpy as np

from . import geometry, occlusion

C0 = 299792458.0
EPS0 = 8.8541878128e-12
# ITU-R P.2040 (Table 3) brick, 1-10 GHz: eps_r = 3.75, sigma = 0.038 S/m
# (frequency independent); the paper's walls are 10 cm of brick (Sec. III-C)
BRICK = dict(eps_r=3.75, sigma=0.038, thickness=0.10)
PEC = "pec"


def reflectors(tri, tol=1e-6):
    """Planes of a triangle soup: list of dict(n, d, tri_index, lo, hi).

    The unit normal of every non-degenerate triangle is taken with its first
    component of magnitude > 1e-9 positive; triangles whose normals and
    offsets agree within tol share a plane."""
    tri = np.asarray(tri, dtype=float).reshape(-1, 3, 3)
    if tri.shape[0] == 0:
        return []
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    ln = np.linalg.norm(nrm, axis=1)
    ok = ln > 0
    nrm[ok] /= ln[ok, None]
    # canonical orientation
    for i in np.nonzero(ok)[0]:
        for c in range(3):
            if abs(nrm[i, c]) > 1e-9:
                if nrm[i, c] < 0:
                    nrm[i] = -nrm[i]
                break
    d = np.einsum("ij,ij->i", nrm, tri[:, 0])
    key = np.round(np.concatenate([nrm, d[:, None]], axis=1) / tol).astype(np.int64)
    out = []
    groups = {}
    for i in np.nonzero(ok)[0]:
        groups.setdefault(tuple(key[i]), []).append(i)
    for k in sorted(groups):
        idx = np.array(groups[k])
        n = nrm[idx[0]]
        pts = tri[idx].reshape(-1, 3)
        out.append(dict(n=n, d=float(np.mean(d[idx])), tri_index=idx, lo=pts.min(axis=0), hi=pts.max(axis=0)))
    return out


def mirror(P, n, d):
    """Image of the points P (..., 3) in the plane n.x = d."""
    P = np.asarray(P, dtype=float)
    h = P @ n - d
    return P - 2.0 * h[..., None] * n


def crossing(A, B, n, d):
    """Where the segments A -> B cross the plane strictly between their end
    points: (Q, ok)."""
    A = np.broadcast_to(np.asarray(A, dtype=float), np.shape(B))
    B = np.asarray(B, dtype=float)
    ha = A @ n - d
    hb = B @ n - d
    ok = ((ha > 0) & (hb < 0)) | ((ha < 0) & (hb > 0))
    t = np.where(ok, ha / np.where(ok, ha - hb, 1.0), 0.0)
    return A + t[:, None] * (B - A), ok


def on_reflector(tri, refl, Q):
    """Does each point Q (on the reflector's plane) lie on one of its
    triangles?  (A short segment through Q along the normal, tested against
    the reflector's own triangles.)"""
    Q = np.asarray(Q, dtype=float).reshape(-1, 3)
    inside = np.all((Q >= refl["lo"] - 1e-9) & (Q <= refl["hi"] + 1e-9), axis=1)
    hit = np.zeros(Q.shape[0], dtype=bool)
    i = np.nonzero(inside)[0]
    if i.size:
        n = refl["n"]
        tri = np.asarray(tri, dtype=float).reshape(-1, 3, 3)[refl["tri_index"]]
        hit[i] = occlusion.segments_vs_triangles(tri, Q[i] - 1e-3 * n, Q[i] + 1e-3 * n)
    return hit


def slab_coefficients(cos_t, f, material):
    """Plane-wave reflection coefficients (R_perp, R_par) of the wall at
    incidence cosines cos_t and frequency f (Hz), time factor e^{+jwt}.

    Half-space interface with eta = eps_r - j sigma/(w eps0) and
    c = sqrt(eta - sin^2):  r_perp = (cos - c)/(cos + c),
    r_par = (eta cos - c)/(eta cos + c); a slab of thickness t has the
    internal phase q = k t c and sums its internal reflections:
    R = r (1 - e^{-2jq}) / (1 - r^2 e^{-2jq}).  The root c is taken with
    a negative imaginary part (a wave decaying into the wall).  A perfect
    conductor has R_perp = -1, R_par = +1."""
    cos_t = np.asarray(cos_t, dtype=float)
    if material == PEC:
        return -np.ones(cos_t.shape, complex), np.ones(cos_t.shape, complex)
    w = 2 * np.pi * f
    eta = material["eps_r"] - 1j * material["sigma"] / (w * EPS0)
    sin2 = 1.0 - cos_t ** 2
    c = np.sqrt(eta - sin2 + 0j)
    c = np.where(c.imag > 0, -c, c)
    r_perp = (cos_t - c) / (cos_t + c)
    r_par = (eta * cos_t - c) / (eta * cos_t + c)
    t = material["thickness"]
    if not np.isfinite(t):
        return r_perp, r_par
    ph = np.exp(-2j * (w / C0) * t * c)
    return (r_perp * (1 - ph) / (1 - r_perp ** 2 * ph), r_par * (1 - ph) / (1 - r_par ** 2 * ph))


def slab_transmission(cos_t, f, material):
    """Plane-wave transmission coefficients (T_perp, T_par) of the slab
    (used only to check the reflection coefficients by energy balance):
    T = (1 - r^2) e^{-jq} / (1 - r^2 e^{-2jq}) relative to the unperturbed
    wave's phase at the slab's entry face."""
    cos_t = np.asarray(cos_t, dtype=float)
    w = 2 * np.pi * f
    eta = material["eps_r"] - 1j * material["sigma"] / (w * EPS0)
    c = np.sqrt(eta - (1.0 - cos_t ** 2) + 0j)
    c = np.where(c.imag > 0, -c, c)
    q = (w / C0) * material["thickness"] * c
    out = []
    for r in ((cos_t - c) / (cos_t + c), (eta * cos_t - c) / (eta * cos_t + c)):
        out.append((1 - r ** 2) * np.exp(-1j * q) / (1 - r ** 2 * np.exp(-2j * q)))
    return tuple(out)


def wall_basis(s_in, s_out, n):
    """(e_perp, e_par_in, e_par_out, cos_t) of a reflection with incident and
    reflected ray directions s_in, s_out (rows) on a plane of normal n."""
    cr = np.cross(s_in, n)
    cn = np.linalg.norm(cr, axis=1)
    alt = geometry._any_perp(np.broadcast_to(n, s_in.shape))
    ep = np.where((cn > 1e-12)[:, None], cr / np.maximum(cn, 1e-300)[:, None], alt)
    return ep, np.cross(ep, s_in), np.cross(ep, s_out), np.abs(s_in @ n)


def reflect_vectors(v, basis, Rp, Rl):
    """R_perp (v.e_perp) e_perp + R_par (v.e_par_in) e_par_out, rows."""
    ep, ei, eo, _ = basis
    a = np.einsum("ij,ij->i", v, ep) * Rp
    b = np.einsum("ij,ij->i", v, ei) * Rl
    return a[:, None] * ep + b[:, None] * eo


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def classify(scene, T, R, inside, opts, visibility=True):
    """Every one-bounce wall path: list of (key, record).  Keys:
    ("w", p) wall only; ("wb", p, body, path) wall then body; ("bw", p,
    body, path) body then wall, with body = ("s", i) or ("c", i) and path =
    ("c", side, ell) or ("r",).  Records hold the wall point Q_w, the wall
    basis, the body record (from the image source, or to the image
    receiver) and the validity after the visibility tests (skipped with
    visibility=False).  The wall-only path tests every body, like the direct
    ray; the other paths' legs test the other bodies when bodies_occlude.
    Wall-fed body paths take the primary creeping paths (no encirclements).
    With lit_branch off (creeping fields only) the wall-only path and the
    body reflections are left out, as the direct ray is."""
    tri = scene.get("tri")
    if tri is None or len(tri) == 0:
        return []
    T = np.asarray(T, dtype=float)
    n_rx = R.shape[0]
    Tb = np.broadcast_to(T, R.shape)
    bodies = [("s", i, b) for i, b in enumerate(scene["spheres"])] + \
             [("c", i, b) for i, b in enumerate(scene["cylinders"])]
    out = []

    def gate(valid, legs, bodies_too):
        if not visibility:
            return valid
        for a0, a1, skip in legs:
            idx = np.nonzero(valid)[0]
            if idx.size:
                blk = occlusion.segments_blocked(scene, a0[idx], a1[idx], skip=skip, bodies=bodies_too)
                valid[idx[blk]] = False
        return valid

    for p, rf in enumerate(reflectors(tri)):
        n, d = rf["n"], rf["d"]
        if T @ n - d == 0:
            continue
        Ti = mirror(T, n, d)
        Tib = np.broadcast_to(Ti, R.shape)
        # wall only: the image source's ray T' -> R crosses the plane on the reflector
        Qw, ok = crossing(Tib, R, n, d)
        ok &= ~inside & bool(opts["lit_branch"])
        ok[ok] = on_reflector(tri, rf, Qw[ok])
        ok = gate(ok, [(Tb, Qw, None), (Qw, R, None)], True)
        s_in = _unit(Qw - Tb)
        out.append((("w", p), dict(kind="wall", valid=ok, Qw=Qw, basis=wall_basis(s_in, _unit(R - Qw), n),
                                   s_i=np.linalg.norm(Qw - Tb, axis=1), s_r=np.linalg.norm(R - Qw, axis=1))))
        Ri = mirror(R, n, d)
        for kind, i, b in bodies:
            bkey = (kind, i)
            for first in ("wb", "bw"):
                src, rcv = (Ti, R) if first == "wb" else (T, Ri)
                if kind == "s":
                    C, a = b[:3], b[3]
                    recs = [(("c", s, 0), geometry.sphere_creeping(src, C, a, rcv, s, 0)) for s in (+1, -1)]
                    if opts["lit_branch"]:
                        recs.append((("r",), geometry.sphere_reflection(src, C, a, rcv)))
                else:
                    plan = geometry.cylinder_plan(src, b, rcv)
                    recs = [(("c", s, 0), geometry.cylinder_creeping(src, b, rcv, s, 0, plan)) for s in (+1, -1)]
                    if opts["lit_branch"]:
                        recs.append((("r",), geometry.cylinder_reflection(src, b, rcv, plan)))
                for pkey, rec in recs:
                    valid = np.asarray(rec["valid"], bool) & ~inside
                    caus = np.zeros(n_rx, bool)
                    if rec["kind"] == "creep":
                        caus = valid & (np.abs(rec["rho_perp"]) < opts["caustic_guard"])
                        valid &= ~caus
                        Qb_in, Qb_out = rec["Q1"], rec["Q2"]
                    else:
                        Qb_in = Qb_out = rec["Q"]
                    if first == "wb":
                        Qw, cr = crossing(Tib, Qb_in, n, d)
                    else:
                        Qw, cr = crossing(Qb_out, Ri, n, d)
                    valid &= cr
                    valid[valid] = on_reflector(tri, rf, Qw[valid])
                    if first == "wb":
                        legs = [(Tb, Qw, None), (Qw, Qb_in, bkey), (Qb_out, R, bkey)]
                        s_in, s_out = _unit(Qw - Tb), _unit(Qb_in - Qw)
                    else:
                        legs = [(Tb, Qb_in, bkey), (Qb_out, Qw, bkey), (Qw, R, None)]
                        s_in, s_out = _unit(Qw - Qb_out), _unit(R - Qw)
                    valid = gate(valid, legs, opts["bodies_occlude"])
                    out.append(((first, p, bkey, pkey), dict(kind=first, valid=valid, caustic=caus, Qw=Qw,
                                                              basis=wall_basis(s_in, s_out, n), body=rec)))
    return out


def add_field(acc, wall_paths, T, dip, amp, f, material, mode="em"):
    """Adds every valid wall path's field at frequency f to acc [3, n]."""
    from . import field as F
    k = 2 * np.pi * f / C0
    for key, rec in wall_paths:
        idx = np.nonzero(rec["valid"])[0]
        if not idx.size:
            continue
        basis = tuple(b[idx] for b in rec["basis"])
        Rp, Rl = slab_coefficients(basis[3], f, material)
        if rec["kind"] == "wall":
            pp, _ = F._incident(T, rec["Qw"][idx], dip, amp, k)
            s = rec["s_i"][idx] + rec["s_r"][idx]
            v = reflect_vectors(pp, basis, Rp, Rl)
            acc[:, idx] += (v * (np.exp(-1j * k * s) / s)[:, None]).T
            continue
        body = rec["body"]
        if rec["kind"] == "wb":
            # the wave arriving at the body is the wall-reflected one; the body
            # record's lengths are measured from the image source
            pp, _ = F._incident(T, rec["Qw"][idx], dip, amp, k)
            inc = reflect_vectors(pp, basis, Rp, Rl)
            if body["kind"] == "creep":
                F._add_creeping(acc, body, idx, None, dip, amp, k, mode, inc=inc)
            else:
                F._add_reflection(acc, body, idx, None, dip, amp, k, mode, inc=inc)
        else:
            # the body's field at the image receiver, reflected at the wall
            part = np.zeros_like(acc)
            if body["kind"] == "creep":
                F._add_creeping(part, body, idx, T, dip, amp, k, mode)
            else:
                F._add_reflection(part, body, idx, T, dip, amp, k, mode)
            acc[:, idx] += reflect_vectors(part[:, idx].T, basis, Rp, Rl).T

"""Coherent receiver field of Eqs. (1)-(4), FP64 oracle.

Test infrastructure (see ``oracle/__init__``).

For every receiver R and frequency f (k = 2 pi f / c, time factor e^{+jwt}):

    E(R) = U_LOS E^i(R)
         + sum_bodies [ U^r E^r(R) + sum_{side, ell} U^d E^d_{side, ell}(R) ]

* E^i(P) = A (p - (p.s)s) e^{-jks}/s, the ray field of a Hertzian dipole p
  at the source T (s = |P - T|, s-hat the direction T -> P).
* E^r: Eq. (3) with the UTD reflection dyadic
  R = e_perp e_perp R_s + e_par^i e_par^r R_h,
  R_p = -sqrt(-4/xi^L) e^{-j (xi^L)^3/12} B_p(xi^L, X^L),
  xi^L = -2 m cos(th_i), X^L = 2 k L^r cos^2(th_i), L^r = s^i s^r/(s^i+s^r).
* E^d: Eq. (4) with the transfer dyadic T = b1 b2 T_s + n1 n2 T_h,
  T_p = -sqrt(m(Q1) m(Q2)) sqrt(2/k) B_p(xi^d, X^d) e^{-jkt},
  xi^d = int m/rho_g dt, X^d = k L^d (xi^d)^2 / (2 m(Q1) m(Q2)),
  L^d = s^i s^d/(s^i + s^d), m = (k rho_g / 2)^{1/3}.
* B_p(xi, X) = p*_p(xi) + e^{-j pi/4} (1 - F(X)) / (2 sqrt(pi) xi).
* Each U is 1 when every segment of the path misses the triangles and the
  other bodies (the line of sight also tests every body).  A receiver inside
  a body gets E = 0.  A creeping path on a sphere whose receiver lies within
  ``caustic_guard`` of the source axis (|rho_perp| small, the axial caustic
  where the ray field is singular) is dropped and the receiver flagged.

With ``caustic_uniform`` the creeping paths of a sphere that meet on the
source axis in pairs, both visible, are summed by the uniform formula of
``oracle/caustic`` instead (finite on the axis); a path left without its
partner is still dropped within ``caustic_guard`` of the axis.

``mode='soft'`` or ``'hard'`` replaces the dipole by a scalar point source
u^i = e^{-jks}/s and keeps only that polarisation; the exact-series checks of
the oracle use it.
"""
import numpy as np

from . import caustic, fock, geometry, occlusion, walls

C0 = 299792458.0

FLAG_INSIDE = 1
FLAG_CAUSTIC = 2
FLAG_LOS = 4


def _opts(opts):
    o = dict(l_enc=0, bodies_occlude=True, lit_branch=True, caustic_guard=1e-6, walls=None,
             caustic_uniform=False)
    if opts:
        o.update(opts)
    return o


def _scene(scene):
    sc = dict(tri=None, spheres=np.zeros((0, 4)), cylinders=np.zeros((0, 5)))
    if scene:
        for k, v in scene.items():
            sc[k] = v
    sc["spheres"] = np.asarray(sc["spheres"], dtype=float).reshape(-1, 4)
    sc["cylinders"] = np.asarray(sc["cylinders"], dtype=float).reshape(-1, 5)
    if sc["tri"] is not None:
        sc["tri"] = np.asarray(sc["tri"], dtype=float).reshape(-1, 3, 3)
    return sc


def inside_mask(scene, R):
    ins = np.zeros(R.shape[0], dtype=bool)
    for cx, cy, cz, a in scene["spheres"]:
        ins |= np.sum((R - np.array([cx, cy, cz])) ** 2, axis=1) <= a * a
    for cx, cy, z0, h, a in scene["cylinders"]:
        ins |= ((R[:, 0] - cx) ** 2 + (R[:, 1] - cy) ** 2 <= a * a) & (R[:, 2] >= z0) & (R[:, 2] <= z0 + h)
    return ins


def source_inside(scene, T):
    return bool(inside_mask(scene, np.asarray(T, dtype=float)[None, :])[0])


def classify(scene, T, R, opts=None, visibility=True):
    """All frequency-independent path data and the visibility decisions
    (``visibility=False`` skips the occlusion tests: every geometrically
    valid path counts as visible and the line of sight as blocked; used when
    the decisions are taken from an earlier call)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return _classify(scene, T, R, opts, visibility)


def _classify(scene, T, R, opts, visibility=True):
    o = _opts(opts)
    sc = _scene(scene)
    T = np.asarray(T, dtype=float)
    R = np.asarray(R, dtype=float).reshape(-1, 3)
    n = R.shape[0]
    inside = inside_mask(sc, R)
    flags = np.where(inside, FLAG_INSIDE, 0).astype(np.uint8)
    Tb = np.broadcast_to(T, R.shape)
    if visibility:
        los = ~occlusion.segments_blocked(sc, Tb, R, skip=None, bodies=True) & ~inside
    else:
        los = np.zeros(n, dtype=bool)
    flags |= np.where(los, FLAG_LOS, 0).astype(np.uint8)
    paths = []
    pairs = []
    uniform = bool(o["caustic_uniform"])
    bodies = [("s", i, b) for i, b in enumerate(sc["spheres"])] + [("c", i, b) for i, b in enumerate(sc["cylinders"])]
    for kind, i, b in bodies:
        if kind == "s":
            C, a = b[:3], b[3]
            recs = [(("c", s, l), geometry.sphere_creeping(T, C, a, R, s, l))
                    for s in (+1, -1) for l in range(o["l_enc"] + 1)]
            if o["lit_branch"]:
                recs.append((("r",), geometry.sphere_reflection(T, C, a, R)))
        else:
            plan = geometry.cylinder_plan(T, b, R)
            recs = [(("c", s, l), geometry.cylinder_creeping(T, b, R, s, l, plan))
                    for s in (+1, -1) for l in range(o["l_enc"] + 1)]
            if o["lit_branch"]:
                recs.append((("r",), geometry.cylinder_reflection(T, b, R, plan)))
        for key, rec in recs:
            valid = rec["valid"] & ~inside
            if rec["kind"] == "creep" and not (uniform and kind == "s"):
                caus = valid & (np.abs(rec["rho_perp"]) < o["caustic_guard"])
                flags |= np.where(caus, FLAG_CAUSTIC, 0).astype(np.uint8)
                valid &= ~caus
            if rec["kind"] == "creep":
                segs = [(Tb, rec["Q1"]), (rec["Q2"], R)]
            else:
                segs = [(Tb, rec["Q"]), (rec["Q"], R)]
            for p0, p1 in (segs if visibility else ()):
                idx = np.nonzero(valid)[0]
                if idx.size:
                    blk = occlusion.segments_blocked(sc, p0[idx], p1[idx], skip=(kind, i),
                                                     bodies=o["bodies_occlude"])
                    valid[idx[blk]] = False
            rec["valid"] = valid
            paths.append(((kind, i) + key, rec))
        if uniform and kind == "s":
            pairs += _pair_up(T, b[:3], b[3], R, dict(recs), o)
            for key, rec in recs:
                if rec["kind"] != "creep":
                    continue
                caus = rec["valid"] & ~rec["paired"] & (np.abs(rec["rho_perp"]) < o["caustic_guard"])
                flags |= np.where(caus, FLAG_CAUSTIC, 0).astype(np.uint8)
                rec["valid"] = rec["valid"] & ~caus
    wall_paths = []
    if o["walls"] is not None:
        # one specular bounce on the scene's planes, alone and feeding the bodies
        wall_paths = walls.classify(sc, T, R, inside, o, visibility)
        for key, rec in wall_paths:
            if "caustic" in rec:
                flags |= np.where(rec["caustic"], FLAG_CAUSTIC, 0).astype(np.uint8)
    return dict(los=los, inside=inside, flags=flags, paths=paths, walls=wall_paths, n=n, pairs=pairs)


def _pair_up(T, C, a, R, recs, o):
    """The caustic pairs of one sphere whose paths are both visible; their
    paths are marked ``paired`` (left out of the per-ray sum)."""
    for key, rec in recs.items():
        if rec["kind"] == "creep":
            rec["paired"] = np.zeros(R.shape[0], dtype=bool)
    rear = caustic.rear_mask(T, C, R)
    out = []
    for side_rear in (True, False):
        for kn, kf in caustic.pair_keys(o["l_enc"], side_rear):
            near, far = recs[("c",) + kn], recs[("c",) + kf]
            sel = near["valid"] & far["valid"] & (rear == side_rear)
            idx = np.nonzero(sel)[0]
            if idx.size:
                near["paired"][idx] = True
                far["paired"][idx] = True
                out.append((C, a, near, far, idx, side_rear))
    return out


def n_rx_frozen(frozen):
    return np.asarray(frozen["los"]).shape[0]


def _incident(T, P, dipole, amp, k):
    """Ray field of the dipole at points P: A (p - (p.s)s) e^{-jks}/s."""
    v = P - T
    s = np.sqrt(np.einsum("ij,ij->i", v, v))
    sh = v / s[:, None]
    pp = dipole[None, :] - (sh @ dipole)[:, None] * sh
    return amp * pp, s


def field(scene, tx, rx, freqs, opts=None, mode="em", frozen=None, return_info=False, return_abs=False):
    """E[f, c, n] (mode 'em') or u[f, n] (mode 'soft'/'hard'), complex128.

    ``frozen``: the classification returned by an earlier call (``return_info``)
    whose visibility decisions are reused; only the geometry is recomputed.
    This is how finite-difference gradients hold the masks fixed.
    ``return_abs``: also return A[f, n] = sum over the receiver's ray
    contributions of their magnitudes ||E_path||_2 (the scale against which
    the rounding error of a coherent sum is bounded per receiver).
    """
    o = _opts(opts)
    sc = _scene(scene)
    T = np.asarray(tx["pos"], dtype=float)
    dip = np.asarray(tx.get("dipole", (0.0, 0.0, 1.0)), dtype=float)
    amp = float(tx.get("amplitude", 1.0))
    R = np.asarray(rx, dtype=float).reshape(-1, 3)
    freqs = np.atleast_1d(np.asarray(freqs, dtype=float))
    info = classify(sc, T, R, o, visibility=frozen is None)
    if frozen is not None and o["caustic_uniform"]:
        raise ValueError("caustic_uniform takes its pairs from the visibility decisions: no frozen classification")
    if frozen is not None:
        info["los"] = frozen["los"]
        info["inside"] = frozen["inside"]
        info["flags"] = frozen["flags"]
        fz = dict(frozen["paths"])
        for key, rec in info["paths"]:
            rec["valid"] = fz[key]["valid"]
        fw = dict(frozen.get("walls", []))
        for key, rec in info["walls"]:
            rec["valid"] = fw[key]["valid"] if key in fw else np.zeros(n_rx_frozen(frozen), bool)
    n = R.shape[0]
    scalar = mode in ("soft", "hard")
    out = np.zeros((freqs.size, n) if scalar else (freqs.size, 3, n), dtype=complex)
    absum = np.zeros((freqs.size, n))
    for fi, f in enumerate(freqs):
        k = 2 * np.pi * f / C0
        acc = out[fi]
        if o["lit_branch"]:
            idx = np.nonzero(info["los"])[0]
            if idx.size:
                if scalar:
                    s = np.linalg.norm(R[idx] - T, axis=1)
                    acc[idx] += np.exp(-1j * k * s) / s
                    absum[fi, idx] += 1.0 / s
                else:
                    pp, s = _incident(T, R[idx], dip, amp, k)
                    acc[:, idx] += (pp * (np.exp(-1j * k * s) / s)[:, None]).T
                    absum[fi, idx] += np.linalg.norm(pp, axis=1) / s
        for key, rec in info["paths"]:
            use = rec["valid"] & ~rec["paired"] if "paired" in rec else rec["valid"]
            idx = np.nonzero(use)[0]
            if not idx.size:
                continue
            part = np.zeros_like(acc) if return_abs else acc
            if rec["kind"] == "creep":
                _add_creeping(part, rec, idx, T, dip, amp, k, mode)
            else:
                _add_reflection(part, rec, idx, T, dip, amp, k, mode)
            if return_abs:
                acc += part
                absum[fi] += np.abs(part) if scalar else np.linalg.norm(part, axis=0)
        for C, a, near, far, idx, rear in info["pairs"]:
            part = np.zeros_like(acc) if return_abs else acc
            caustic.add_pair(part, T, C, a, R, near, far, idx, rear, dip, amp, k, mode)
            if return_abs:
                acc += part
                absum[fi] += np.abs(part) if scalar else np.linalg.norm(part, axis=0)
        if info["walls"]:
            if scalar:
                raise ValueError("wall reflections need mode 'em'")
            for key, rec in info["walls"]:
                part = np.zeros_like(acc) if return_abs else acc
                walls.add_field(part, [(key, rec)], T, dip, amp, f, o["walls"], mode)
                if return_abs:
                    acc += part
                    absum[fi] += np.linalg.norm(part, axis=0)
    res = (out,)
    if return_info:
        res += (info,)
    if return_abs:
        res += (absum,)
    return res[0] if len(res) == 1 else res


def _take(rec, name, idx):
    v = rec[name]
    return v[idx] if np.ndim(v) > 0 else np.full(idx.shape, v)


def _add_creeping(acc, rec, idx, T, dip, amp, k, mode, inc=None):
    """Adds the creeping field of the paths idx of rec into acc.  ``inc``:
    the amplitude-weighted incident polarisation vectors at Q1 when the
    wave arriving there is not the source's own (a wall reflection); the
    record's s_i is then the distance from the equivalent (image) source."""
    rho_g = _take(rec, "rho_g", idx)
    sI, t, sD = _take(rec, "s_i", idx), _take(rec, "t", idx), _take(rec, "s_d", idx)
    m = (k * rho_g / 2) ** (1.0 / 3.0)
    xi = m * t / rho_g
    L = sI * sD / (sI + sD)
    X = k * L * xi ** 2 / (2 * m * m)
    q = np.sqrt(k * L / 2) / m
    pref = -m * np.sqrt(2 / k)
    S = _take(rec, "S", idx)
    phase = np.exp(-1j * k * (sI + t + sD))
    if mode in ("soft", "hard"):
        Tp = pref * fock.shadow_B(xi, X, q, mode == "hard")
        acc[idx] += Tp * S * phase / sI
        return
    Ts = pref * fock.shadow_B(xi, X, q, False)
    Th = pref * fock.shadow_B(xi, X, q, True)
    if inc is None:
        pp, s = _incident(T, rec["Q1"][idx], dip, amp, k)
    else:
        pp = inc
    es = np.einsum("ij,ij->i", pp, rec["b1"][idx]) * Ts
    eh = np.einsum("ij,ij->i", pp, rec["n1"][idx]) * Th
    common = S * phase / sI
    acc[:, idx] += ((es * common)[:, None] * rec["b2"][idx] + (eh * common)[:, None] * rec["n2"][idx]).T


def _add_reflection(acc, rec, idx, T, dip, amp, k, mode, inc=None):
    """Adds the reflected field of the paths idx of rec into acc (``inc`` as
    for _add_creeping, at the reflection point)."""
    rho_g = rec["rho_g"][idx]
    cos_i = rec["cos_i"][idx]
    sI, sR = rec["s_i"][idx], rec["s_r"][idx]
    m = (k * rho_g / 2) ** (1.0 / 3.0)
    xi = -2 * m * cos_i
    L = sI * sR / (sI + sR)
    X = 2 * k * L * cos_i ** 2
    q = np.sqrt(k * L / 2) / m
    rho1, rho2 = rec["rho1"][idx], rec["rho2"][idx]
    # R_p sqrt(rho1 rho2/((rho1+s)(rho2+s))) = 2 sqrt(rho1/(-xi)) Rbar_p sqrt(rho2/((rho1+s)(rho2+s)))
    rho1_over_mxi = rec["rho1_over_cos"][idx] / (2 * m)
    spread = 2 * np.sqrt(rho1_over_mxi) * np.sqrt(rho2 / ((rho1 + sR) * (rho2 + sR)))
    phase = np.exp(-1j * k * (sI + sR))
    if mode in ("soft", "hard"):
        Rb = fock.lit_Rbar(xi, X, q, mode == "hard")
        acc[idx] += Rb * spread * phase / sI
        return
    Rs = fock.lit_Rbar(xi, X, q, False)
    Rh = fock.lit_Rbar(xi, X, q, True)
    if inc is None:
        pp, s = _incident(T, rec["Q"][idx], dip, amp, k)
    else:
        pp = inc
    es = np.einsum("ij,ij->i", pp, rec["eperp"][idx]) * Rs
    eh = np.einsum("ij,ij->i", pp, rec["epar_i"][idx]) * Rh
    common = spread * phase / sI
    acc[:, idx] += ((es * common)[:, None] * rec["eperp"][idx] + (eh * common)[:, None] * rec["epar_r"][idx]).T

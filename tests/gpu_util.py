"""Helpers shared by the GPU tests: run the HIP library through its binding
and compare against the oracle on the same float32-rounded inputs.

Field parity is receiver-exact: the library also returns its visibility
decisions (``path_masks``), the oracle evaluates the field with exactly those
decisions (its ``frozen`` classification), and the two fields are compared at
every receiver.  Separately, the library's decisions are compared with the
oracle's own (FP32 watertight BVH test against FP64 Moller-Trumbore); every
decision that differs must be a grazing one: moving the segment's end points
by DELTA_GRAZE metres flips the oracle's own decision.
"""
import numpy as np

import workloads as W

TOL = {0: 1e-4, 1: 1e-10}
# end-point displacement (m) within which a differing visibility decision
# counts as grazing: FP32 rounding of coordinates of about 10 m is ~1e-6 m
DELTA_GRAZE = 2e-5


def _dev_inputs(cfg, rx, freqs):
    import torch
    sc = cfg["scene"]
    sph = torch.from_numpy(np.ascontiguousarray(sc["spheres"], np.float32).reshape(-1, 4)).cuda()
    cyl = torch.from_numpy(np.ascontiguousarray(sc["cylinders"], np.float32).reshape(-1, 5)).cuda()
    rxt = torch.from_numpy(np.ascontiguousarray(rx, np.float32).reshape(-1, 3)).cuda()
    ft = torch.from_numpy(np.ascontiguousarray(freqs, np.float64)).cuda()
    return sph, cyl, rxt, ft


def set_walls(scene, walls):
    """Library wall material from the oracle's description (dict or PEC)."""
    from oracle import walls as OW
    if walls == OW.PEC:
        scene.set_wall_material(perfect_conductor=True)
    else:
        scene.set_wall_material(walls["eps_r"], walls["sigma"], walls["thickness"])


def run_library(cfg, precision=0, rx=None, freqs=None, masks=False, walls=None, **kw):
    """(E complex128 [nf, 3, n], flags [n]) and, with masks=True, the
    library's per-(body, receiver) path masks [nb, n] for the same inputs
    (and, with walls, its wall masks [n, n_planes] as a fourth item).
    ``walls``: the oracle's wall material (dict or PEC) to switch wall
    reflections on."""
    import torch

    import paper_2310_10578_amd as utd
    sc = cfg["scene"]
    scene = utd.Scene(sc.get("tri"))
    rx = cfg["rx"] if rx is None else rx
    freqs = cfg["freqs"] if freqs is None else freqs
    sph, cyl, rxt, ft = _dev_inputs(cfg, rx, freqs)
    tx = cfg["tx"]
    src = utd.make_source(tx["pos"], tx["dipole"], tx["amplitude"])
    if walls is not None:
        set_walls(scene, walls)
    E, flags = utd.smooth_field(scene, sph, cyl, src, rxt, ft, precision=precision,
                                wall_reflections=walls is not None, **kw)
    if masks:
        mk, fm = utd.path_masks(scene, sph, cyl, src, rxt, precision=precision, **kw)
        if walls is not None:
            wm = utd.wall_masks(scene, sph, cyl, src, rxt, precision=precision, **kw)
    torch.cuda.synchronize()
    out = E.cpu().numpy().astype(np.complex128), flags.cpu().numpy()
    if masks:
        fm = fm.cpu().numpy()
        assert np.array_equal(fm, out[1] & ~np.uint8(2 | 64)), "path_masks flags differ from the field call's"
        out = out + (mk.cpu().numpy(),)
        if walls is not None:
            out = out + (wm.cpu().numpy().view(np.uint64),)
    scene.close()
    return out


def run_oracle(cfg, rx=None, freqs=None, opts=None, frozen=None, absum=False):
    from oracle import field
    sc, tx, r = W.to_oracle(cfg["scene"], cfg["tx"], cfg["rx"] if rx is None else rx)
    freqs = cfg["freqs"] if freqs is None else freqs
    return field.field(sc, tx, r, freqs, opts=opts, return_info=True, frozen=frozen, return_abs=absum)


def normwise(Eg, Eo):
    """Per frequency ||E_gpu - E_ref||_2 / ||E_ref||_2 over all receivers and components."""
    num = np.sqrt(np.sum(np.abs(Eg - Eo) ** 2, axis=(1, 2)))
    den = np.sqrt(np.sum(np.abs(Eo) ** 2, axis=(1, 2)))
    return num / den


def path_keys(n_sph, n_cyl, l_enc, lit_branch):
    """(oracle path key, body index, mask bit) for every path the library
    can set: bodies spheres first, creeping bit 2 ell + (side < 0), reflection 6."""
    out = []
    for b in range(n_sph + n_cyl):
        body = ("s", b) if b < n_sph else ("c", b - n_sph)
        for s in (+1, -1):
            for ell in range(l_enc + 1):
                out.append((body + ("c", s, ell), b, 2 * ell + (1 if s < 0 else 0)))
        if lit_branch:
            out.append((body + ("r",), b, 6))
    return out


def wall_keys(n_planes, n_sph, n_cyl):
    """(oracle wall-path key, plane, bit) for every bit of the library's wall masks."""
    out = []
    for p in range(n_planes):
        out.append((("w", p), p, 0))
        for b in range(n_sph + n_cyl):
            body = ("s", b) if b < n_sph else ("c", b - n_sph)
            for k, (first, path) in enumerate([("wb", ("c", 1, 0)), ("wb", ("c", -1, 0)), ("wb", ("r",)),
                                               ("bw", ("c", 1, 0)), ("bw", ("c", -1, 0)), ("bw", ("r",))]):
                out.append(((first, p, body, path), p, 1 + 6 * b + k))
    return out


def frozen_from_library(cfg, flags, mask, opts=None, wmask=None):
    """The library's decisions in the oracle's classification layout (wall
    paths from its wall masks when given)."""
    o = dict(l_enc=0, lit_branch=True)
    o.update(opts or {})
    ns = np.asarray(cfg["scene"]["spheres"]).reshape(-1, 4).shape[0]
    nc = np.asarray(cfg["scene"]["cylinders"]).reshape(-1, 5).shape[0]
    dead = (flags & (1 | 8 | 16 | 32)) != 0
    paths = [(key, dict(valid=((mask[b] >> bit) & 1).astype(bool) & ~dead))
             for key, b, bit in path_keys(ns, nc, o["l_enc"], o["lit_branch"])]
    fz = dict(los=(flags & 4) != 0, inside=(flags & 1) != 0, flags=flags.copy(), paths=paths)
    if wmask is not None:
        wm = np.asarray(wmask, np.uint64)
        fz["walls"] = [(key, dict(valid=((wm[:, p] >> np.uint64(bit)) & np.uint64(1)).astype(bool) & ~dead))
                       for key, p, bit in wall_keys(wm.shape[1], ns, nc)]
    return fz


def wall_decision_mismatches(cfg, rx, flags, wmask, walls, opts=None, delta=DELTA_GRAZE, n_try=12, seed=0):
    """The library's wall decisions against the oracle's own.  Returns
    (n_differing, n_not_grazing); a difference is grazing when moving the
    receiver by delta in some direction flips the oracle's own decision."""
    from oracle import field
    o = dict(l_enc=0, lit_branch=True, bodies_occlude=True, caustic_guard=1e-6)
    o.update(opts or {})
    o["walls"] = walls
    sc, tx, R = W.to_oracle(cfg["scene"], cfg["tx"], rx)
    T = np.asarray(tx["pos"], float)
    info = field.classify(sc, T, R, o)
    ns = np.asarray(cfg["scene"]["spheres"]).reshape(-1, 4).shape[0]
    nc = np.asarray(cfg["scene"]["cylinders"]).reshape(-1, 5).shape[0]
    dead = (flags & (1 | 8 | 16 | 32)) != 0
    own = dict(info["walls"])
    wm = np.asarray(wmask, np.uint64)
    diff = []
    for key, p, bit in wall_keys(wm.shape[1], ns, nc):
        g = ((wm[:, p] >> np.uint64(bit)) & np.uint64(1)).astype(bool) & ~dead
        vo = np.asarray(own[key]["valid"], bool) if key in own else np.zeros(len(g), bool)
        for i in np.nonzero(g != vo)[0]:
            diff.append((i, key, vo[i]))
    rng = np.random.default_rng(seed)
    n_not = 0
    for i, key, base in diff:
        flipped = False
        for _ in range(n_try):
            u = rng.standard_normal(3)
            Rp = R[i] + delta * u / np.linalg.norm(u)
            inf2 = dict(field.classify(sc, T, Rp[None, :], o)["walls"])
            if key in inf2 and bool(inf2[key]["valid"][0]) != base:
                flipped = True
                break
        n_not += 0 if flipped else 1
    return len(diff), n_not


def _segments(info, key, idx, T, R):
    rec = dict(info["paths"])[key]
    if rec["kind"] == "creep":
        return [(np.broadcast_to(T, (idx.size, 3)), rec["Q1"][idx]), (rec["Q2"][idx], R[idx])]
    return [(np.broadcast_to(T, (idx.size, 3)), rec["Q"][idx]), (rec["Q"][idx], R[idx])]


def _grazing(sc, segs, skip, bodies, delta, n_try=16, seed=0):
    """Per path: does moving the end points of its legs by up to delta flip
    the oracle's visibility of the path?"""
    from oracle import occlusion
    rng = np.random.default_rng(seed)
    n = segs[0][0].shape[0]
    base = np.ones(n, bool)
    for p0, p1 in segs:
        base &= ~occlusion.segments_blocked(sc, p0, p1, skip=skip, bodies=bodies)
    seen_other = np.zeros(n, bool)
    for _ in range(n_try):
        vis = np.ones(n, bool)
        for p0, p1 in segs:
            u = rng.standard_normal(p0.shape)
            v = rng.standard_normal(p1.shape)
            u *= delta / np.linalg.norm(u, axis=1, keepdims=True)
            v *= delta / np.linalg.norm(v, axis=1, keepdims=True)
            vis &= ~occlusion.segments_blocked(sc, p0 + u, p1 + v, skip=skip, bodies=bodies)
        seen_other |= vis != base
    return seen_other


def decision_mismatches(cfg, rx, flags, mask, info, opts=None):
    """Compares the library's decisions with the oracle's own.  Returns
    (n_los, n_path, n_not_grazing): the differing line-of-sight and path
    decisions, and how many of them are not grazing."""
    from oracle import field
    o = dict(l_enc=0, lit_branch=True, bodies_occlude=True)
    o.update(opts or {})
    sc, tx, R = W.to_oracle(cfg["scene"], cfg["tx"], rx)
    T = np.asarray(tx["pos"], float)
    # the oracle's geometric path existence (no visibility tests)
    geo = dict(field.classify(sc, T, R, o, visibility=False)["paths"])
    dead = (flags & (1 | 8 | 16 | 32)) != 0
    n_not = 0
    los_g = (flags & 4) != 0
    los_o = np.asarray(info["los"], bool)
    dl = np.nonzero(los_g != los_o)[0]
    if dl.size:
        segs = [(np.broadcast_to(T, (dl.size, 3)), R[dl])]
        n_not += int((~_grazing(sc, segs, None, True, DELTA_GRAZE)).sum())
    n_path = 0
    ns = np.asarray(cfg["scene"]["spheres"]).reshape(-1, 4).shape[0]
    nc = np.asarray(cfg["scene"]["cylinders"]).reshape(-1, 5).shape[0]
    recs = dict(info["paths"])
    for key, b, bit in path_keys(ns, nc, o["l_enc"], o["lit_branch"]):
        g = ((mask[b] >> bit) & 1).astype(bool) & ~dead
        vo = np.asarray(recs[key]["valid"], bool)
        d = np.nonzero(g != vo)[0]
        if not d.size:
            continue
        n_path += d.size
        # a path that the oracle's geometry does not have is a classification
        # difference, not a visibility one: never accepted
        exists = np.asarray(geo[key]["valid"], bool)[d]
        segs = _segments(info, key, d, T, R)
        gz = _grazing(sc, segs, key[:2], o["bodies_occlude"], DELTA_GRAZE) & exists
        n_not += int((~gz).sum())
    return int(dl.size), n_path, n_not


def per_receiver(Eg, Eo, A):
    """Per receiver and frequency: |dE| / A (A = sum of the receiver's path
    magnitudes, the componentwise scale), and reading 14's metric
    |dE| / max(|E_ref|, 1e-3 RMS_f)."""
    d = np.linalg.norm(Eg - Eo, axis=1)
    comp = d / np.maximum(A, 1e-300)
    ref = np.linalg.norm(Eo, axis=1)
    rms = np.sqrt(np.mean(ref ** 2, axis=1, keepdims=True))
    r14 = d / np.maximum(ref, 1e-3 * rms)
    return comp, r14


def parity(cfg, precision, rx=None, freqs=None, opts=None, name="", r14_bound=None, check_decisions=True,
           max_mismatch=0.02, sample=None, tol=None, lib=None, sens=None, nw_tol=None, walls=None):
    """Receiver-exact parity of the library against the oracle.

    1. The library's field against the oracle evaluated with the library's
       own decisions: normwise per frequency and per receiver (|dE| <= TOL
       times the sum of the receiver's path magnitudes) within the contract
       tolerance, at every receiver; reading 14's per-receiver metric reported
       (and bounded when r14_bound is given).
    2. The library's decisions against the oracle's: the inside and caustic
       flags exactly; line-of-sight flags and path bits may differ only where
       grazing, on at most max_mismatch of the receivers.
    ``sample``: indices of the receivers the oracle recomputes (the library
    runs on all of them, in the launch configuration of the full size).
    ``lib``: the library's (E, flags, masks) when already computed.
    ``sens``: per (frequency, receiver) the oracle's own change under a few
    ulps of receiver displacement (ill-conditioned receivers); the
    per-receiver bound is then TOL times the path magnitudes plus 4 sens.
    ``nw_tol``: the normwise bound when it differs from the per-receiver TOL.
    ``walls``: the oracle's wall material (dict or PEC): wall reflections on
    in both, the library's wall decisions frozen into the oracle too.
    Returns a dict of the measured numbers."""
    opts = dict(opts or {})
    tol = TOL[precision] if tol is None else tol
    nw_tol = tol if nw_tol is None else nw_tol
    rx = cfg["rx"] if rx is None else rx
    freqs = cfg["freqs"] if freqs is None else freqs
    if lib is None:
        lib = run_library(cfg, precision, rx=rx, freqs=freqs, masks=True, walls=walls, **opts)
    Eg, fg, mk = lib[:3]
    wm = lib[3] if len(lib) > 3 else None
    if sample is not None:
        Eg, fg, mk, rx = Eg[:, :, sample], fg[sample], mk[:, sample], rx[sample]
        wm = wm[sample] if wm is not None else None
    frozen = frozen_from_library(cfg, fg, mk, opts, wmask=wm)
    oopts = dict(opts, walls=walls) if walls is not None else opts
    Eo, _, A = run_oracle(cfg, rx=rx, freqs=freqs, opts=oopts, frozen=frozen, absum=True)
    nw = normwise(Eg, Eo)
    comp, r14 = per_receiver(Eg, Eo, A)
    res = dict(normwise=nw, comp=comp, r14=r14, flags=fg, mask=mk, E=Eg, Eo=Eo, A=A, rx=rx)
    msg = "%s p%d: normwise max %.2e, per-receiver componentwise max %.2e, reading-14 max %.2e" % (
        name, precision, nw.max(), comp.max(), r14.max())
    if check_decisions:
        _, info = run_oracle(cfg, rx=rx, freqs=freqs[:1], opts=oopts)
        n_los, n_path, n_not = decision_mismatches(cfg, rx, fg, mk, info, opts)
        if wm is not None:
            n_w, n_w_not = wall_decision_mismatches(cfg, rx, fg, wm, walls, opts)
            n_path += n_w
            n_not += n_w_not
        res.update(n_los=n_los, n_path=n_path, n_not_grazing=n_not, info=info)
        msg += "; decisions differing from the oracle's: %d line-of-sight, %d paths (%d not grazing) of %d rx" % (
            n_los, n_path, n_not, fg.size)
    print(msg, flush=True)
    assert np.all(nw <= nw_tol), nw
    if sens is None:
        assert comp.max() <= tol, comp.max()
    else:
        assert np.all(np.linalg.norm(Eg - Eo, axis=1) <= tol * A + 4.0 * sens)
    if r14_bound is not None:
        assert r14.max() <= r14_bound, r14.max()
    if check_decisions:
        np.testing.assert_array_equal(fg & 3, info["flags"] & 3)
        assert n_not == 0
        assert (n_los + n_path) <= max_mismatch * fg.size
    return res

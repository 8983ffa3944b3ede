"""The batched entry point (many frames, one persistent launch replayed as a
HIP graph) against per-frame calls of utd_smooth_field and against the
oracle.

Per frame the batched kernel accumulates in the order of the single-frame
kernels, so the two agree to floating-point contraction differences:
normwise <= 1e-6 (FP32) and <= 1e-12 (FP64); flags must match exactly."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _crowd(n_frames=10, n_pop=16, rx_range=(40, 700)):
    return W.crowd(n_frames=n_frames, n_pop=n_pop, rx_range=rx_range, edge=0.5)


def _to_dev(cfg):
    import torch
    d = dict(body_off=torch.from_numpy(cfg["body_off"]).cuda(), rx_off=torch.from_numpy(cfg["rx_off"]).cuda(),
             cyl=torch.from_numpy(np.ascontiguousarray(cfg["cylinders"], np.float32)).cuda(),
             rx=torch.from_numpy(np.ascontiguousarray(cfg["rx"], np.float32)).cuda(),
             freqs=torch.from_numpy(np.asarray(cfg["freqs"], np.float64)).cuda())
    return d


def _batched(cfg, precision, scene, d, **kw):
    import torch

    import paper_2310_10578_amd as utd
    tx = cfg["tx"]
    src = utd.make_source(tx["pos"], tx["dipole"], tx["amplitude"])
    E, fl = utd.smooth_field_batched(scene, d["body_off"], d["cyl"], d["rx_off"], d["rx"], src, d["freqs"],
                                     precision=precision, **kw)
    torch.cuda.synchronize()
    return E.cpu().numpy().astype(np.complex128), fl.cpu().numpy()


def _frames(cfg, E, fl, bo=None, ro=None):
    bo = cfg["body_off"] if bo is None else bo
    ro = cfg["rx_off"] if ro is None else ro
    nf = len(cfg["freqs"])
    for f in range(len(bo) - 1):
        n = ro[f + 1] - ro[f]
        blk = E[3 * nf * ro[f]: 3 * nf * ro[f + 1]].reshape(nf, 3, n)
        yield f, cfg["cylinders"][bo[f]:bo[f + 1]], cfg["rx"][ro[f]:ro[f + 1]], blk, fl[ro[f]:ro[f + 1]]


def _single(cfg, scene, cyl, rx, precision, **kw):
    import torch

    import paper_2310_10578_amd as utd
    tx = cfg["tx"]
    src = utd.make_source(tx["pos"], tx["dipole"], tx["amplitude"])
    c = torch.from_numpy(np.ascontiguousarray(cyl, np.float32).reshape(-1, 5)).cuda()
    r = torch.from_numpy(np.ascontiguousarray(rx, np.float32).reshape(-1, 3)).cuda()
    f = torch.from_numpy(np.asarray(cfg["freqs"], np.float64)).cuda()
    E, fl = utd.smooth_field(scene, None, c, src, r, f, precision=precision, **kw)
    torch.cuda.synchronize()
    return E.cpu().numpy().astype(np.complex128), fl.cpu().numpy()


TOL = {0: 1e-6, 1: 1e-12}


@pytest.mark.parametrize("tile,bpc", [(64, 2), (128, 4), (256, 1)])
@pytest.mark.parametrize("precision", [0, 1])
def test_batched_equals_per_frame(precision, tile, bpc):
    import paper_2310_10578_amd as utd
    cfg = _crowd()
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    utd.batched_config(tile, bpc)
    E, fl = _batched(cfg, precision, scene, d)
    worst = 0.0
    for f, cyl, rx, blk, flb in _frames(cfg, E, fl):
        if rx.shape[0] == 0:
            continue
        Es, fls = _single(cfg, scene, cyl, rx, precision)
        np.testing.assert_array_equal(flb, fls)
        den = np.linalg.norm(Es)
        worst = max(worst, np.linalg.norm(blk - Es) / den if den > 0 else np.linalg.norm(blk))
    print("batched vs per-frame p%d tile %d: worst frame %.2e" % (precision, tile, worst), flush=True)
    assert worst <= TOL[precision]
    scene.close()


@pytest.mark.parametrize("precision", [1, 0])
def test_batched_vs_oracle(precision):
    """Two frames of the crowd against the oracle (frame with the most
    cylinders and one other)."""
    import paper_2310_10578_amd as utd
    cfg = _crowd(n_frames=6, rx_range=(40, 300))
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    utd.batched_config(128, 4)
    E, fl = _batched(cfg, precision, scene, d)
    nb = np.diff(cfg["body_off"])
    import torch
    from gpu_util import parity
    src = utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"])
    for f in sorted({int(np.argmax(nb)), 1}):
        _, cyl, rx, blk, flb = list(_frames(cfg, E, fl))[f]
        one = dict(scene=dict(tri=cfg["tri"], spheres=np.zeros((0, 4), np.float32), cylinders=cyl),
                   tx=cfg["tx"], rx=rx, freqs=cfg["freqs"])
        # the oracle takes the decisions of a per-frame call on the same frame
        mk, _ = utd.path_masks(scene, None, torch.from_numpy(np.ascontiguousarray(cyl)).cuda(), src,
                               torch.from_numpy(np.ascontiguousarray(rx)).cuda(), precision=precision)
        torch.cuda.synchronize()
        parity(one, precision, lib=(blk, flb, mk.cpu().numpy()),
               name="batched frame %d (%d cylinders)" % (f, cyl.shape[0]))
    scene.close()


def test_empty_and_malformed_frames():
    """Frames with no cylinders or no receivers, and offsets that run past
    the arrays or decrease, are clamped on the device to the running maximum
    within [0, n]: the output equals per-frame calls on the clamped frames."""
    import torch

    import paper_2310_10578_amd as utd
    cfg = _crowd(n_frames=5, rx_range=(30, 200))
    n_cyl, n_rx = cfg["cylinders"].shape[0], cfg["rx"].shape[0]
    bo = cfg["body_off"].copy()
    ro = cfg["rx_off"].copy()
    bo[2] = bo[1]                          # frame 1 without cylinders
    ro[4] = ro[3]                          # frame 3 without receivers
    bo_bad = bo.copy()
    ro_bad = ro.copy()
    bo_bad[3] = bo[1] - 1                  # decreasing -> clamped to the running max
    bo_bad[5] = n_cyl + 7                  # past the array -> n_cyl
    ro_bad[5] = n_rx + 11
    clamp = lambda a, n: np.maximum.accumulate(np.clip(a, 0, n))
    bo_ok, ro_ok = clamp(bo_bad, n_cyl), clamp(ro_bad, n_rx)
    bo_ok[0] = ro_ok[0] = 0
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    d["body_off"] = torch.from_numpy(bo_bad).cuda()
    d["rx_off"] = torch.from_numpy(ro_bad).cuda()
    utd.batched_config(64, 2)
    E, fl = _batched(cfg, 0, scene, d)
    for f, cyl, rx, blk, flb in _frames(cfg, E, fl, bo_ok, ro_ok):
        if rx.shape[0] == 0:
            continue
        Es, fls = _single(cfg, scene, cyl, rx, 0)
        np.testing.assert_array_equal(flb, fls)
        assert np.linalg.norm(blk - Es) <= 1e-6 * np.linalg.norm(Es)
    # no frames / no receivers / no frequencies: nothing to do
    e0 = torch.zeros(0, dtype=torch.complex64, device="cuda")
    src = utd.make_source(cfg["tx"]["pos"])
    z = torch.zeros(1, dtype=torch.int64, device="cuda")
    utd.smooth_field_batched(scene, z, d["cyl"], z, d["rx"][:0], src, d["freqs"], out=e0)
    scene.close()


def test_graph_replay_reads_fresh_device_data():
    """The captured graph is replayed while the arguments repeat: moving the
    cylinders in place between calls (eager work and synchronisations in
    between) changes every replay's result exactly as per-frame calls on the
    moved cylinders."""
    import torch

    import paper_2310_10578_amd as utd
    cfg = _crowd(n_frames=4, rx_range=(30, 200))
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    utd.batched_config(128, 2)
    src = utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"])
    out = torch.empty(3 * len(cfg["freqs"]) * cfg["rx"].shape[0], dtype=torch.complex64, device="cuda")
    flags = torch.empty(cfg["rx"].shape[0], dtype=torch.uint8, device="cuda")
    base = d["cyl"].clone()
    for rep in range(3):
        d["cyl"].copy_(base)
        d["cyl"][:, 0] += 0.01 * rep
        torch.cuda.synchronize()
        utd.smooth_field_batched(scene, d["body_off"], d["cyl"], d["rx_off"], d["rx"], src, d["freqs"], out=out,
                                 flags=flags)
        torch.cuda.synchronize()
        E = out.cpu().numpy().astype(np.complex128)
        fl = flags.cpu().numpy()
        moved = dict(cfg)
        moved["cylinders"] = d["cyl"].cpu().numpy()
        for f, cyl, rx, blk, flb in _frames(moved, E, fl):
            if rx.shape[0] == 0:
                continue
            Es, fls = _single(moved, scene, cyl, rx, 0)
            np.testing.assert_array_equal(flb, fls)
            assert np.linalg.norm(blk - Es) <= 1e-6 * np.linalg.norm(Es)
    scene.close()


def test_capture_into_caller_graph():
    """Inside torch.cuda.graph capture the call records its launches into the
    caller's graph; every replay matches the eager result."""
    import torch

    import paper_2310_10578_amd as utd
    cfg = _crowd(n_frames=4, rx_range=(30, 200))
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    utd.batched_config(128, 2)
    src = utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"])
    n = cfg["rx"].shape[0]
    out = torch.empty(3 * len(cfg["freqs"]) * n, dtype=torch.complex64, device="cuda")
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    utd.smooth_field_batched(scene, d["body_off"], d["cyl"], d["rx_off"], d["rx"], src, d["freqs"], out=out,
                             flags=flags)
    torch.cuda.synchronize()
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            utd.smooth_field_batched(scene, d["body_off"], d["cyl"], d["rx_off"], d["rx"], src, d["freqs"],
                                     out=out, flags=flags, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    # a larger call grows the library's workspace; the captured graph still
    # points into the old one, which must stay alive
    big = _crowd(n_frames=12, rx_range=(2000, 4000))
    db = _to_dev(big)
    Eb, _ = utd.smooth_field_batched(scene, db["body_off"], db["cyl"], db["rx_off"], db["rx"], src, db["freqs"])
    torch.cuda.synchronize()
    for rep in range(2):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    del Eb
    scene.close()


def _compare_frames(cfg, E, fl, scene, precision, frames=None, tol=None, **kw):
    """Per-frame calls of utd_smooth_field against the batched blocks: flags
    exactly, fields normwise within tol (default TOL).  Returns the worst."""
    tol = TOL[precision] if tol is None else tol
    worst = 0.0
    for f, cyl, rx, blk, flb in _frames(cfg, E, fl):
        if (frames is not None and f not in frames) or rx.shape[0] == 0:
            continue
        Es, fls = _single(cfg, scene, cyl, rx, precision, **kw)
        np.testing.assert_array_equal(flb, fls)
        den = np.linalg.norm(Es)
        worst = max(worst, np.linalg.norm(blk - Es) / den if den > 0 else np.linalg.norm(blk))
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("kw", [dict(l_enc=2), dict(lit_branch=False), dict()])
@pytest.mark.parametrize("precision", [0, 1])
def test_batched_second_body_group_and_options(precision, kw):
    """Frames with up to 64 cylinders (so the persistent kernel's second
    group of 32 bodies runs, and with l_enc = 2 -- seven paths per pair -- its
    LDS candidate queue drains after almost every body), encirclements and
    creeping-only fields, at the autotuned tile shape 256 x 3: equal to
    per-frame calls."""
    import paper_2310_10578_amd as utd
    cfg = _crowd(n_frames=8, n_pop=64, rx_range=(200, 900))
    nb = np.diff(cfg["body_off"])
    assert nb.max() > 32
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    utd.batched_config(256, 3)
    E, fl = _batched(cfg, precision, scene, d, **kw)
    worst = _compare_frames(cfg, E, fl, scene, precision, **kw)
    print("batched vs per-frame p%d %s, up to %d cylinders: worst frame %.2e" % (precision, kw, nb.max(), worst),
          flush=True)
    scene.close()


def test_crowd_full_size_sampled_frames():
    """Config 4 at full size (256 frames of the 2.0e5-triangle room, 0..64
    cylinders, 1k..64k receivers, 8 frequencies, FP32) in the bench's launch
    configuration (tile 256 x 3): the frames with the most cylinders and the
    most receivers and two more, against per-frame calls (flags exact,
    fields within 1e-6); two of them also against the oracle on 200 sampled
    receivers each, evaluated with the per-frame call's decisions."""
    import paper_2310_10578_amd as utd
    from gpu_util import parity
    cfg = W.crowd()
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    utd.batched_config(256, 3)
    E, fl = _batched(cfg, 0, scene, d)
    nb, nr = np.diff(cfg["body_off"]), np.diff(cfg["rx_off"])
    frames = sorted({int(np.argmax(nb)), int(np.argmax(nr)), int(np.argmax(nb * (nr > 30000))), 17})
    worst = _compare_frames(cfg, E, fl, scene, 0, frames=frames)
    print("crowd full size: frames %s (cylinders %s, receivers %s) vs per-frame: worst %.2e" % (
        frames, nb[frames].tolist(), nr[frames].tolist(), worst), flush=True)
    allf = list(_frames(cfg, E, fl))
    rng = np.random.default_rng(11)
    for f in frames[:2]:
        _, cyl, rx, blk, flb = allf[f]
        one = dict(scene=dict(tri=cfg["tri"], spheres=np.zeros((0, 4), np.float32), cylinders=cyl),
                   tx=cfg["tx"], rx=rx, freqs=cfg["freqs"])
        idx = np.sort(rng.choice(rx.shape[0], 200, replace=False))
        import torch
        src = utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"])
        mk, _ = utd.path_masks(scene, None, torch.from_numpy(np.ascontiguousarray(cyl)).cuda(), src,
                               torch.from_numpy(np.ascontiguousarray(rx)).cuda())
        torch.cuda.synchronize()
        parity(one, 0, sample=idx, lib=(blk, flb, mk.cpu().numpy()), name="crowd frame %d (%d cylinders)" % (
            f, cyl.shape[0]))
    scene.close()


def test_batched_invalid_inputs():
    """Invalid device inputs in the batched call: a non-finite receiver (its
    field zero, flagged), an invalid cylinder in one frame (that frame's
    field zero and flagged, the other frames unchanged) and an invalid
    frequency (zero at that frequency, every receiver flagged); never a
    non-finite field."""
    import torch

    import paper_2310_10578_amd as utd
    cfg = _crowd(n_frames=4, n_pop=16, rx_range=(60, 200))
    scene = utd.Scene(cfg["tri"])
    utd.batched_config(128, 2)
    d = _to_dev(cfg)
    E0, f0 = _batched(cfg, 0, scene, d)
    utd.input_status()
    bo, ro = cfg["body_off"], cfg["rx_off"]
    fb = int(np.argmax(np.diff(bo) > 0))                   # a frame with cylinders
    bad_cyl = d["cyl"].clone()
    bad_cyl[bo[fb], 4] = -0.1
    rx_bad = d["rx"].clone()
    rx_bad[ro[2] + 1, 1] = float("nan")
    d2 = dict(d, cyl=bad_cyl, rx=rx_bad)
    E, fl = _batched(cfg, 0, scene, d2)
    assert np.isfinite(E).all()
    assert utd.input_status() == utd.BAD_BODY | utd.BAD_RX
    nf = len(cfg["freqs"])
    for f in range(len(bo) - 1):
        blk = slice(3 * nf * ro[f], 3 * nf * ro[f + 1])
        if f == fb:
            assert np.all(E[blk] == 0) and np.all(fl[ro[f]:ro[f + 1]] & utd.FLAG_BAD_BODY)
        elif f == 2:
            i = ro[2] + 1
            assert fl[i] & utd.FLAG_INVALID_RX
            E3 = E[blk].reshape(nf, 3, -1)
            assert np.all(E3[:, :, 1] == 0)
        else:
            np.testing.assert_array_equal(E[blk], E0[blk])
    freqs = d["freqs"].clone()
    freqs[1] = -2e9
    E, fl = _batched(cfg, 0, scene, dict(d, freqs=freqs))
    assert np.isfinite(E).all() and np.all(fl & utd.FLAG_BAD_FREQ)
    assert utd.input_status() == utd.BAD_FREQ
    E3 = E.reshape(-1)
    for f in range(len(bo) - 1):
        n = ro[f + 1] - ro[f]
        blk = E3[3 * nf * ro[f]: 3 * nf * ro[f + 1]].reshape(nf, 3, n)
        ref = E0[3 * nf * ro[f]: 3 * nf * ro[f + 1]].reshape(nf, 3, n)
        assert np.all(blk[1] == 0)
        np.testing.assert_array_equal(blk[[0] + list(range(2, nf))], ref[[0] + list(range(2, nf))])
    scene.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_receiver_layouts(precision):
    """The kernel visits each frame's receivers in a spatial (Morton cell)
    order and writes every result back to the receiver's own place: frames
    whose receivers are one repeated point, a vertical line, a 3-D block, a
    single receiver, and a large shuffled grid with non-finite receivers
    mixed in equal per-frame calls (flags exactly, fields within TOL)."""
    import torch

    import paper_2310_10578_amd as utd
    base = _crowd(n_frames=6, n_pop=24, rx_range=(40, 60))
    rng = np.random.default_rng(5)
    layouts = [
        np.tile([[3.1, 2.2, 1.2]], (300, 1)),
        np.stack([np.full(257, 6.4), np.full(257, 5.1), np.linspace(0.1, 2.9, 257)], 1),
        np.stack(np.meshgrid(np.linspace(0.5, 9.5, 12), np.linspace(0.5, 7.5, 10), np.linspace(0.3, 2.7, 9),
                             indexing="ij"), -1).reshape(-1, 3),
        np.array([[4.4, 1.3, 1.0]]),
        np.stack(np.meshgrid(np.linspace(0.05, 9.95, 80), np.linspace(0.05, 7.95, 64), [1.2],
                             indexing="ij"), -1).reshape(-1, 3),
        rng.uniform([0, 0, 0], [10, 8, 3], (2000, 3)),
    ]
    layouts[4] = layouts[4][rng.permutation(layouts[4].shape[0])]
    layouts[4][[7, 1000, 4000]] = [[np.nan, 1.0, 1.0], [np.inf, 2.0, 1.2], [1.0, -np.inf, 0.5]]
    rx = np.concatenate(layouts).astype(np.float32)
    rx_off = np.concatenate([[0], np.cumsum([len(a) for a in layouts])]).astype(np.int64)
    cfg = dict(base, rx=rx, rx_off=rx_off)
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    utd.batched_config(256, 3)
    E, fl = _batched(cfg, precision, scene, d)
    assert np.isfinite(E).all()
    worst = _compare_frames(cfg, E, fl, scene, precision)
    bad = rx_off[4] + np.array([7, 1000, 4000])
    assert np.all(fl[bad] & utd.FLAG_INVALID_RX)
    utd.input_status()
    print("receiver layouts p%d: worst frame %.2e" % (precision, worst), flush=True)
    scene.close()


def test_batched_many_frequencies_accumulate_in_place():
    """With many frequencies the per-block field scratch would pass its size
    cap, and the lanes accumulate in the output directly: 160 frequencies in
    FP64 at tile 256 x 3 equal per-frame calls."""
    import paper_2310_10578_amd as utd
    cfg = _crowd(n_frames=3, n_pop=12, rx_range=(300, 700))
    cfg = dict(cfg, freqs=np.linspace(2.0e9, 6.0e9, 160))
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    utd.batched_config(256, 3)
    E, fl = _batched(cfg, 1, scene, d)
    worst = _compare_frames(cfg, E, fl, scene, 1)
    print("160 frequencies FP64 in place: worst frame %.2e" % worst, flush=True)
    scene.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_source_leg_profiles(precision):
    """The batched kernel decides a creeping path's source-side leg from a
    per-(frame, cylinder, side) profile of the fan of legs to the tangent
    line, falling back to the leg's own test where a height is undecided or
    the profile does not exist.  A dense set of low boxes with the source
    below the tops of many of them (many cuts per fan: some profiles
    overflow, many heights sit near cut boundaries), cylinders of random
    heights and a source at several heights: equal to per-frame calls, which
    test every leg."""
    import paper_2310_10578_amd as utd
    rng = np.random.default_rng(23)
    Lx, Ly = 10.0, 8.0
    boxes = []
    for _ in range(120):
        sz = rng.uniform([0.1, 0.1, 0.2], [0.6, 0.6, 1.8])
        x0, y0 = rng.uniform(0, Lx - sz[0]), rng.uniform(0, Ly - sz[1])
        boxes.append((np.array([x0, y0, 0.0]), np.array([x0 + sz[0], y0 + sz[1], sz[2]])))
    tri = np.concatenate([W.room_shell(0.5)] + [W.box_triangles(lo, hi) for lo, hi in boxes]).astype(np.float32)
    cyls, rxs, bo, ro = [], [], [0], [0]
    for f in range(6):
        nb = int(rng.integers(8, 40))
        c = np.stack([rng.uniform(0.5, Lx - 0.5, nb), rng.uniform(0.5, Ly - 0.5, nb), np.zeros(nb),
                      rng.uniform(0.8, 2.2, nb), rng.uniform(0.12, 0.3, nb)], 1)
        nr = int(rng.integers(300, 1500))
        r = np.stack([rng.uniform(0, Lx, nr), rng.uniform(0, Ly, nr), rng.uniform(0.3, 2.0, nr)], 1)
        cyls.append(c)
        rxs.append(r)
        bo.append(bo[-1] + nb)
        ro.append(ro[-1] + nr)
    scene = utd.Scene(tri)
    for tz in (0.6, 1.4, 2.6):
        cfg = dict(tri=tri, cylinders=np.concatenate(cyls).astype(np.float32), rx=np.concatenate(rxs).astype(np.float32),
                   body_off=np.array(bo, np.int64), rx_off=np.array(ro, np.int64),
                   tx=dict(pos=np.array([4.7, 3.3, tz], np.float32), dipole=np.array([0.2, 0.3, 0.9], np.float32),
                           amplitude=1.0),
                   freqs=np.array([2.4e9, 5.0e9]))
        d = _to_dev(cfg)
        utd.batched_config(256, 3)
        E, fl = _batched(cfg, precision, scene, d, l_enc=1)
        worst = _compare_frames(cfg, E, fl, scene, precision, l_enc=1)
        print("source-leg profiles p%d, source at %.1f m: worst frame %.2e" % (precision, tz, worst), flush=True)
    scene.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_result_independent_of_tile_shape(precision):
    """Each receiver's field is summed by one lane in a fixed order (direct
    ray, then per group of 32 bodies its creeping paths and its
    reflections), and every visibility decision depends on its own path
    only, so the tile shape and the workgroups per CU must not change a
    single bit of the output: frames of up to 64 cylinders (two body
    groups), l_enc = 0 and 2."""
    import torch

    import paper_2310_10578_amd as utd
    cfg = _crowd(n_frames=8, n_pop=64, rx_range=(100, 1500))
    scene = utd.Scene(cfg["tri"])
    d = _to_dev(cfg)
    for l_enc in (0, 2):
        ref = None
        for tile, bpc in ((256, 3), (128, 6), (64, 8), (256, 1)):
            utd.batched_config(tile, bpc)
            E, fl = _batched(cfg, precision, scene, d, l_enc=l_enc)
            if ref is None:
                ref = (E, fl)
                continue
            assert np.array_equal(fl, ref[1]), (tile, bpc, l_enc)
            assert np.array_equal(E, ref[0]), (tile, bpc, l_enc, float(np.max(np.abs(E - ref[0]))))
    utd.batched_config(256, 3)
    torch.cuda.synchronize()
    scene.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_tile_cull_receiver_by_receiver(precision):
    """The tile-box cull skips a body for a whole tile only when no receiver
    of the tile could carry one of its paths.  Receivers fill a band of
    heights around the cylinders' tops, with the source above them, so that
    many tiles' boxes straddle the heights where a cylinder's paths start or
    stop existing; every receiver's field must equal that of per-frame calls
    (which test every pair), receiver by receiver."""
    import torch

    import paper_2310_10578_amd as utd
    rng = np.random.default_rng(97)
    Lx, Ly = 10.0, 8.0
    tri = np.concatenate([W.room_shell(0.5)] + [W.box_triangles(np.array([x, y, 0.0]), np.array([x + 0.4, y + 0.4, 0.8]))
                                                for x, y in ((2.0, 2.0), (7.0, 5.0), (4.5, 6.5))]).astype(np.float32)
    cyls, rxs, bo, ro = [], [], [0], [0]
    for f in range(4):
        nb = int(rng.integers(16, 48))
        c = np.stack([rng.uniform(0.5, Lx - 0.5, nb), rng.uniform(0.5, Ly - 0.5, nb), np.zeros(nb),
                      rng.uniform(1.0, 1.6, nb), rng.uniform(0.12, 0.3, nb)], 1)
        nr = int(rng.integers(2000, 5000))
        r = np.stack([rng.uniform(0, Lx, nr), rng.uniform(0, Ly, nr), rng.uniform(0.9, 1.7, nr)], 1)
        cyls.append(c)
        rxs.append(r)
        bo.append(bo[-1] + nb)
        ro.append(ro[-1] + nr)
    cfg = dict(tri=tri, cylinders=np.concatenate(cyls).astype(np.float32), rx=np.concatenate(rxs).astype(np.float32),
               body_off=np.array(bo, np.int64), rx_off=np.array(ro, np.int64),
               tx=dict(pos=np.array([5.1, 3.9, 2.1], np.float32), dipole=np.array([0.3, 0.1, 0.9], np.float32),
                       amplitude=1.0),
               freqs=np.array([2.4e9, 3.6e9, 5.8e9]))
    scene = utd.Scene(tri)
    d = _to_dev(cfg)
    # the two calls sum each receiver's paths in different orders: rounding
    # differences, relative to the receiver's field or to 1 % of the frame's
    # RMS field (a factor of up to 100 for weak receivers) -- about 1e-7
    # (FP32) and 1e-13 (FP64) before that factor; a dropped or added path
    # changes a receiver by far more (1e-3 and up)
    tol = {0: 1e-5, 1: 1e-9}[precision]
    for kw in (dict(), dict(l_enc=1)):
        utd.batched_config(256, 3)
        E, fl = _batched(cfg, precision, scene, d, **kw)
        worst = 0.0
        for f, cyl, rx, blk, flb in _frames(cfg, E, fl):
            Es, fls = _single(cfg, scene, cyl, rx, precision, **kw)
            np.testing.assert_array_equal(flb, fls)
            mag = np.sqrt(np.sum(np.abs(Es) ** 2, axis=(0, 1)))
            diff = np.sqrt(np.sum(np.abs(blk - Es) ** 2, axis=(0, 1)))
            floor = 1e-2 * np.sqrt(np.mean(mag ** 2))
            worst = max(worst, float(np.max(diff / np.maximum(mag, floor))))
        print("tile cull p%d %s: worst receiver %.2e" % (precision, kw, worst), flush=True)
        assert worst <= tol, worst
    torch.cuda.synchronize()
    scene.close()

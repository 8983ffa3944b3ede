"""Throughput of the smooth-surface UTD field evaluation on one MI355X.

A step is one pass of the whole hot path over one batch of the headline
workload, the dynamic crowd: 256 frames of the indoor room (10 x 8 x 3 m,
2.0e5 triangles), 0..64 moving vertical PEC cylinders and 1k..64k receivers
per frame, 8 frequencies in 3.4..3.8 GHz, as one utd_smooth_field_batched
call (body and frequency constants, per-(receiver, body) classification and
geodesics, reflection points, visibility against the BVH and the other
cylinders, Fock evaluation and the coherent field of every (receiver, body,
frequency), FP32 with FP64 path lengths and phase).  Inputs are resident in
HBM before the timed region.

The same JSON line also carries (each timed on its own, after the headline):
  per_frame   the crowd as 256 plain utd_smooth_field calls (batched / plain)
  field       the sphere-plane workload (a = 1 m, 256 x 256 receivers, 64
              frequencies in 1-6 GHz): the field kernel k_field, ALU roofline
  occlusion   the room (32 cylinders, 512 x 512 receivers, 5 and 28 GHz): the
              visibility pass, HBM traffic from the committed counters
  adjoint     the room with 64 cylinders, 128 x 128 receivers, 16 frequencies:
              forward, backward and forward+backward with the saved state
  cpu_baseline the FP64 oracle on a bounded sample of the crowd

``--gpus`` above 1 is refused: this library runs on one GPU.
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 arithmetic operations per (path, frequency) as the field kernels
# execute them (utd_kernels.hip add_path, utd_fock.h fock_kernel; an add or
# a multiply counts 1, an FMA 2, a hardware sin, cos or exp2 1; compares,
# selects, clamps, conversions and fract are not counted):
#   creeping path: Fock arguments 5, transition table (index 3 + degree-4
#     complex Horner 16) 19, regime table (index 2 + degree-4 soft+hard
#     complex Horner 32) 34, combine 12, phase sin/cos 2, phase times the two
#     coefficients 12, accumulation into 3 complex components 24 -> 108
#   reflection: Fock arguments 8, transition 19, regime (index 6 + Horner
#     32) 38, combine 8, e^{-j xi^3/12} 7 and its three complex products 18,
#     sums 4, phase 2, products 12, accumulation 24 -> 140
# Each path also takes 3 FP64 operations per frequency for its phase
# f s_tot / c - n_c / 4 (not counted as FP32).  Per (receiver, frequency):
# the direct ray 14 (sin/cos 2 + 6 FMA), the k^{-1/6} scaling 6.
FLOPS_CREEP = 108
FLOPS_REFL = 140
FLOPS_LOS = 14
FLOPS_RX_SCALE = 6
# Frequency-independent work per candidate path (classification, geodesic or
# reflection point, path constants: steps a2-a4), the lower end of the
# algorithmic per-path figure the method's formula set needs (120-180 FP32
# flops).  The batched kernel does these steps for every (receiver, body)
# pair and each of its 2 (l_enc + 1) creeping paths and its reflection, so
# its algorithmic count is pairs x paths per pair x 120 plus the field of
# the paths that exist and are visible.
FLOPS_PATH_GEOM = 120
# Uniform sum of a sphere's creeping-ray pair at the axial caustic, per
# (pair, frequency): the two rays' Fock coefficients 2 x 84 (the creeping
# count above without its accumulation), J_0..J_3 by their power series to
# the accuracy used (4 x 8 terms x 2) 64, the combination (6 Bessel
# weights, 4 complex interpolations, 9 complex real-weighted sums and the
# 3 x 3 complex accumulation) 218 -> 450; counted against the FP64 rate
# (the Bessel functions and the geometry are FP64).
FLOPS_CAUSTIC_PAIR_FREQ = 450
PEAK_FP64_TFLOPS = 78.6
# MI355X FP32 vector rate: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
# = 78.6 TFLOP/s for the plain FP32 instructions this library is built with
# (packed FP32, which doubles it to the published 157.3, is disabled at
# compile time); both are reported.
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PUBLISHED_TFLOPS = 157.3
PEAK_HBM_GBPS = 8000.0

TRAFFIC_PROFILE = {"sphere_plane": "profiles/counters_k_field_sphere-plane-64f.md",
                   "room": "profiles/counters_k_vis_room-512x512-2f.md",
                   "crowd": "profiles/counters_k_batch_crowd-256f.md"}
VIS_KERNELS = ("utd::k_setup", "utd::k_cand<float", "utd::k_vis<float", "utd::k_rec<float", "utd::k_paths<float")


def kernel_source_digest():
    """SHA-256 over the device sources (names and contents, sorted by name)."""
    import glob
    import hashlib
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2310_10578_amd", "csrc", "*.h")) +
                   glob.glob(os.path.join(ROOT, "paper_2310_10578_amd", "csrc", "*.hip")))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name, kernel_prefix):
    """HBM bytes per launch of a kernel from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE runs, calibrated against a device copy), or
    None when there is none for this workload or the device sources have
    changed since the counters were taken."""
    rel = TRAFFIC_PROFILE.get(workload_name)
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    digest, val = None, None
    with open(os.path.join(ROOT, rel)) as fh:
        for line in fh:
            if line.startswith("kernel_sources_sha256:"):
                digest = line.split(":", 1)[1].strip()
            if line.startswith("traffic_bytes " + kernel_prefix):
                val = float(line.rsplit("=", 1)[1])
    if digest != kernel_source_digest():
        return None
    return val


def _progress(msg):
    """One line on stderr per finished phase (the JSON line stays alone on stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="crowd", choices=["crowd", "sphere_plane", "room", "room_adjoint"],
                    help="headline workload (default: the crowd, batched)")
    ap.add_argument("--secondary", type=int, default=1, help="also time the per-frame, field, occlusion and "
                                                             "adjoint measurements")
    ap.add_argument("--secondary-steps", type=int, default=200, help="timed calls of the field/occlusion workloads")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-frames", type=int, default=16, help="crowd frames in the oracle sample")
    ap.add_argument("--cpu-rx", type=int, default=48, help="receivers per frame in the oracle sample")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this size (HBM counter calibration under a profiler)")
    return ap.parse_args()


def _dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _event_ms(fn, steps, warmup):
    """Average milliseconds per call over `steps` calls after `warmup`,
    bracketed by events on the current stream (the stream the library
    launches on) and device synchronisations."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _kernel_ms(fn, steps, kernel):
    """Average duration of one library kernel class per call, from the
    library's HIP event pairs recorded around each launch on its stream."""
    import paper_2310_10578_amd as utd
    utd.profile_enable(True)
    utd.profile_read()
    for _ in range(steps):
        fn()
    prof = utd.profile_read()
    utd.profile_enable(False)
    ms, n = prof[kernel]
    return ms / max(n, 1), {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}


def _path_flops(census, n_f, n_live):
    """FP32 operations of the field evaluation for a path census."""
    creep, refl, los = census["creeping"], census["reflections"], census["los"]
    return ((creep * FLOPS_CREEP + refl * FLOPS_REFL + los * FLOPS_LOS) + n_live * FLOPS_RX_SCALE) * n_f


def _alu_roofline(flops, kernel_ms, kernel, extra=None):
    achieved = flops / (kernel_ms / 1e3) / 1e12
    r = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
         "frac": achieved / PEAK_FP32_TFLOPS, "frac_of_published_157.3": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
         "kernel": kernel, "kernel_ms": kernel_ms, "flops_per_launch": flops}
    if extra:
        r.update(extra)
    return r


# ---------------------------------------------------------------------------
# the crowd (headline): batched and per-frame
# ---------------------------------------------------------------------------

def crowd_setup():
    import torch

    import paper_2310_10578_amd as utd
    import workloads as W
    cfg = W.crowd()
    d = dict(cfg=cfg, scene=utd.Scene(cfg["tri"]), bo=_dev(cfg["body_off"]), ro=_dev(cfg["rx_off"]),
             cyl=_dev(cfg["cylinders"]), rx=_dev(cfg["rx"]), freqs=_dev(np.asarray(cfg["freqs"], np.float64)),
             src=utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"]))
    n_rx, n_f = d["rx"].shape[0], d["freqs"].shape[0]
    d["out"] = torch.empty((3 * n_f * n_rx,), dtype=torch.complex64, device="cuda:0")
    d["flags"] = torch.empty((n_rx,), dtype=torch.uint8, device="cuda:0")
    nb, nr = np.diff(cfg["body_off"]), np.diff(cfg["rx_off"])
    d["evals"] = int((nb * nr).sum()) * n_f
    return d


def crowd_batched(d, steps, warmup):
    import paper_2310_10578_amd as utd
    from paper_2310_10578_amd.autotune import tune_batched
    tune = tune_batched(d["scene"], d["bo"], d["cyl"], d["ro"], d["rx"], d["src"], d["freqs"], out=d["out"],
                        flags=d["flags"])

    def step():
        utd.smooth_field_batched(d["scene"], d["bo"], d["cyl"], d["ro"], d["rx"], d["src"], d["freqs"],
                                 out=d["out"], flags=d["flags"])

    t0 = time.perf_counter()
    ms = _event_ms(step, steps, warmup)
    wall = time.perf_counter() - t0
    k_ms, per_kernel = _kernel_ms(step, max(2, steps // 2), "batched")
    return ms, wall, k_ms, per_kernel, tune


def crowd_census(d):
    """Path census of every frame (outside any timed region)."""
    import paper_2310_10578_amd as utd
    cfg = d["cfg"]
    bo, ro = cfg["body_off"], cfg["rx_off"]
    tot = dict(creeping=0, reflections=0, los=0, inside=0)
    for f in range(len(bo) - 1):
        if ro[f + 1] == ro[f]:
            continue
        c = utd.path_census(d["scene"], None, d["cyl"][bo[f]:bo[f + 1]], d["src"], d["rx"][ro[f]:ro[f + 1]])
        for k in tot:
            tot[k] += c[k]
    return tot


def crowd_per_frame(d, steps):
    import paper_2310_10578_amd as utd
    cfg = d["cfg"]
    bo, ro = cfg["body_off"], cfg["rx_off"]
    n_f = d["freqs"].shape[0]
    frames = []
    for f in range(len(bo) - 1):
        n = int(ro[f + 1] - ro[f])
        if n == 0:
            continue
        frames.append((d["cyl"][bo[f]:bo[f + 1]], d["rx"][ro[f]:ro[f + 1]],
                       d["out"][3 * n_f * ro[f]: 3 * n_f * ro[f + 1]].view(n_f, 3, n), d["flags"][ro[f]:ro[f + 1]]))

    def per_frame():
        for c, r, o, fl in frames:
            utd.smooth_field(d["scene"], None, c, d["src"], r, d["freqs"], out=o, flags=fl)

    return _event_ms(per_frame, steps, 1)


# ---------------------------------------------------------------------------
# single-call workloads: field kernel (sphere plane), visibility (room)
# ---------------------------------------------------------------------------

def single_setup(name):
    import torch

    import paper_2310_10578_amd as utd
    import workloads as W
    cfg = getattr(W, name)()
    sc = cfg["scene"]
    d = dict(cfg=cfg, scene=utd.Scene(sc.get("tri")), sph=_dev(np.asarray(sc["spheres"], np.float32)),
             cyl=_dev(np.asarray(sc["cylinders"], np.float32)), rx=_dev(cfg["rx"]),
             freqs=_dev(np.asarray(cfg["freqs"], np.float64)),
             src=utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"]))
    n_rx, n_f = d["rx"].shape[0], d["freqs"].shape[0]
    d["n_body"] = d["sph"].shape[0] + d["cyl"].shape[0]
    d["out"] = torch.empty((n_f, 3, n_rx), dtype=torch.complex64, device="cuda:0")
    d["flags"] = torch.empty((n_rx,), dtype=torch.uint8, device="cuda:0")
    d["evals"] = n_rx * max(d["n_body"], 1) * n_f
    return d


def single_step(d):
    import paper_2310_10578_amd as utd
    return lambda: utd.smooth_field(d["scene"], d["sph"], d["cyl"], d["src"], d["rx"], d["freqs"], precision=0,
                                    out=d["out"], flags=d["flags"])


def field_measure(name, steps, warmup):
    """One call per step; the field kernel's roofline (ALU) and the
    visibility pass's time and HBM traffic."""
    import paper_2310_10578_amd as utd
    d = single_setup(name)
    step = single_step(d)
    ms = _event_ms(step, steps, warmup)
    f_ms, per_kernel = _kernel_ms(step, steps, "field")
    census = utd.path_census(d["scene"], d["sph"], d["cyl"], d["src"], d["rx"])
    n_rx, n_f = d["rx"].shape[0], d["freqs"].shape[0]
    flops = _path_flops(census, n_f, n_rx - census["inside"])
    occ_ms = per_kernel.get("occlude", 0.0)
    vis_bytes = [measured_traffic(name, k) for k in VIS_KERNELS]
    vis_bytes = sum(v for v in vis_bytes if v is not None) if any(v is not None for v in vis_bytes) else None
    res = {"workload": d["cfg"]["name"], "evals_per_step": d["evals"], "ms_per_step": ms,
           "evals_per_s": d["evals"] / (ms / 1e3), "kernels_ms_per_step": per_kernel,
           "roofline": _alu_roofline(flops, f_ms, "k_field<float>",
                                     {"traffic": measured_traffic(name, "utd::k_field<float"),
                                      "paths": census["creeping"] + census["reflections"],
                                      "creeping": census["creeping"], "reflections": census["reflections"],
                                      "los_receivers": census["los"]}),
           "visibility": {"ms": occ_ms, "pairs": n_rx * max(d["n_body"], 1),
                          "visible_paths": census["creeping"] + census["reflections"],
                          "hbm_bytes": vis_bytes,
                          "hbm_GBps": (vis_bytes / (occ_ms / 1e3) / 1e9) if (vis_bytes and occ_ms) else None,
                          "frac_of_hbm_peak": (vis_bytes / (occ_ms / 1e3) / 1e9 / PEAK_HBM_GBPS)
                          if (vis_bytes and occ_ms) else None}}
    d["scene"].close()
    return res


def caustic_measure(steps, warmup):
    """The sphere workload with one encirclement (rear and front pairs) and
    the uniform caustic sum, against the same call without it; the pair
    kernels' time and the pairs they summed (counted on the host from the
    library's own visibility masks: both paths of a pair visible)."""
    import paper_2310_10578_amd as utd
    d = single_setup("sphere_plane")
    kw = dict(precision=0, l_enc=1, out=d["out"], flags=d["flags"])
    on = lambda: utd.smooth_field(d["scene"], d["sph"], d["cyl"], d["src"], d["rx"], d["freqs"],
                                  caustic_uniform=True, **kw)
    off = lambda: utd.smooth_field(d["scene"], d["sph"], d["cyl"], d["src"], d["rx"], d["freqs"], **kw)
    ms_on = _event_ms(on, steps, warmup)
    ms_off = _event_ms(off, steps, warmup)
    # per call: the two pair kernels (k_pair, k_caustic) share one timing class
    utd.profile_enable(True)
    utd.profile_read()
    for _ in range(steps):
        on()
    prof = utd.profile_read()
    utd.profile_enable(False)
    k_ms = prof["caustic"][0] / steps
    per_kernel = {k: v[0] / steps for k, v in prof.items() if v[1]}
    mk, _ = utd.path_masks(d["scene"], d["sph"], d["cyl"], d["src"], d["rx"], l_enc=1, caustic_guard=0.0)
    mk = mk.cpu().numpy()
    rx = d["cfg"]["rx"].astype(np.float64)
    T = np.asarray(d["cfg"]["tx"]["pos"], np.float64)
    pairs = 0
    for b, sph in enumerate(np.asarray(d["cfg"]["scene"]["spheres"], np.float64).reshape(-1, 4)):
        rear = (rx - sph[:3]) @ (T - sph[:3]) < 0
        m = mk[b].astype(np.int64)
        both = lambda i, j: ((m >> i) & 1).astype(bool) & ((m >> j) & 1).astype(bool)
        pairs += int(np.sum(rear & both(0, 1)) + np.sum(rear & both(2, 3)) + np.sum(~rear & both(1, 2)))
    n_f = d["freqs"].shape[0]
    flops = pairs * n_f * FLOPS_CAUSTIC_PAIR_FREQ
    achieved = flops / (k_ms / 1e3) / 1e12 if k_ms > 0 else None
    res = {"workload": d["cfg"]["name"] + " l_enc=1 caustic_uniform", "ms_per_step": ms_on,
           "ms_per_step_without": ms_off, "pairs": pairs, "frequencies": n_f,
           "pair_freqs_per_s": pairs * n_f / (k_ms / 1e3) if k_ms > 0 else None,
           "kernels_ms_per_step": per_kernel,
           "roofline": {"bound": "alu", "kernel": "k_pair + k_caustic<float>", "kernel_ms": k_ms,
                        "flops_per_launch": flops, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS if achieved else None}}
    d["scene"].close()
    return res


def adjoint_measure(steps):
    """Forward and backward (loss = sum |E|^2, dL/dE = 2E) on the room with
    64 cylinders, 128 x 128 receivers, 16 frequencies, FP32: the backward from
    scratch (it repeats classification and visibility) and the backward from
    the state a forward call saved (the autograd path)."""
    import paper_2310_10578_amd as utd
    d = single_setup("room_adjoint")
    step = single_step(d)
    step()
    gE = 2 * d["out"]
    fwd = _event_ms(step, steps, 1)
    bwd = _event_ms(lambda: utd.smooth_field_backward(d["scene"], d["sph"], d["cyl"], d["src"], d["rx"], d["freqs"],
                                                      gE), steps, 1)

    def fwd_saved():
        _, _, st = utd.smooth_field_saved(d["scene"], d["sph"], d["cyl"], d["src"], d["rx"], d["freqs"],
                                          out=d["out"], flags=d["flags"])
        st.release()

    fs = _event_ms(fwd_saved, steps, 1)
    _, _, st = utd.smooth_field_saved(d["scene"], d["sph"], d["cyl"], d["src"], d["rx"], d["freqs"], out=d["out"],
                                      flags=d["flags"])
    bs = _event_ms(lambda: utd.smooth_field_backward_saved(st, gE), steps, 1)
    _, kern = _kernel_ms(lambda: utd.smooth_field_backward_saved(st, gE), steps, "backward")
    st.release()
    res = {"workload": d["cfg"]["name"], "evals_per_step": d["evals"], "gradients": 3 + 3 * d["n_body"],
           "fwd_ms": fwd, "bwd_ms": bwd, "bwd_over_fwd": bwd / fwd,
           "fwd_saved_ms": fs, "bwd_saved_ms": bs, "bwd_saved_over_fwd": bs / fwd,
           "fwd_evals_per_s": d["evals"] / (fwd / 1e3), "bwd_saved_evals_per_s": d["evals"] / (bs / 1e3),
           "bwd_saved_kernels_ms_per_step": kern}
    d["scene"].close()
    return res


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the crowd
# ---------------------------------------------------------------------------

def _host_info():
    info = {"python_cpu_count": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
        lines = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines()
        for ln in lines:
            if ln.startswith("Model name") or ln.startswith("CPU(s):") or ln.startswith("Thread(s) per core"):
                info[ln.split(":")[0].strip()] = ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError, ValueError):
        info["machine"] = platform.machine()
    return info


def _oracle_frame(a):
    """Timed: the oracle as it stands (its own visibility decisions).  Then,
    untimed: the same receivers with the library's decisions frozen (the
    error of the GPU result is taken against this one); the difference of
    the two times is the oracle's occlusion time."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import field
    sc, tx, rx, freqs, frozen = a
    t0 = time.perf_counter()
    E_own = field.field(sc, tx, rx, freqs)
    t1 = time.perf_counter()
    E_frz = field.field(sc, tx, rx, freqs, frozen=frozen)
    t2 = time.perf_counter()
    return E_own, E_frz, t1 - t0, max((t1 - t0) - (t2 - t1), 0.0)


def _frozen(mask, flags, n_cyl):
    """The library's decisions (cylinders only, l_enc = 0, reflections on) in
    the oracle's classification layout."""
    dead = (flags & (1 | 8 | 16 | 32)) != 0
    paths = []
    for b in range(n_cyl):
        for s in (+1, -1):
            paths.append((("c", b, "c", s, 0), dict(valid=((mask[b] >> (0 if s > 0 else 1)) & 1).astype(bool) & ~dead)))
        paths.append((("c", b, "r"), dict(valid=((mask[b] >> 6) & 1).astype(bool) & ~dead)))
    return dict(los=(flags & 4) != 0, inside=(flags & 1) != 0, flags=flags.copy(), paths=paths)


def _oracle_frame_k(kt):
    return kt[0], _oracle_frame(kt[1])


def cpu_baseline(d, n_frames, n_rx):
    """The FP64 oracle on a seeded sample of the crowd: n_frames frames with
    cylinders, n_rx receivers of each, all 8 frequencies; one worker process
    per frame on the host's CPU share for one GPU (at most 16), timed
    wall-clock.  Also the FP32 error of the batched result on the sample,
    against the oracle evaluated with the library's own decisions (taken
    from utd_path_masks on each sampled frame), and how many sampled
    receivers' fields differ between those decisions and the oracle's."""
    import multiprocessing as mp

    import paper_2310_10578_amd as utd
    import workloads as W
    cfg = d["cfg"]
    bo, ro = cfg["body_off"], cfg["rx_off"]
    rng = np.random.default_rng(11)
    cand = [f for f in range(len(bo) - 1) if bo[f + 1] > bo[f] and ro[f + 1] - ro[f] >= n_rx]
    frames = sorted(rng.choice(cand, min(n_frames, len(cand)), replace=False).tolist())
    tasks, picks = [], []
    for f in frames:
        idx = np.sort(rng.choice(ro[f + 1] - ro[f], n_rx, replace=False))
        rx_f = cfg["rx"][ro[f]:ro[f + 1]][idx]
        mk, fl = utd.path_masks(d["scene"], None, d["cyl"][bo[f]:bo[f + 1]], d["src"], _dev(rx_f))
        import torch
        torch.cuda.synchronize()
        scene = dict(tri=cfg["tri"], spheres=np.zeros((0, 4), np.float32), cylinders=cfg["cylinders"][bo[f]:bo[f + 1]])
        sc, tx, rx = W.to_oracle(scene, cfg["tx"], rx_f)
        tasks.append((sc, tx, rx, cfg["freqs"], _frozen(mk.cpu().numpy(), fl.cpu().numpy(), int(bo[f + 1] - bo[f]))))
        picks.append((f, idx))
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    procs = max(1, min(share, 16, len(tasks)))
    # the workers are joined, not terminated: a worker killed by a signal
    # can hang in a profiler's exit handler when this runs under one
    pool = mp.get_context("fork").Pool(procs)
    try:
        parts = [None] * len(tasks)
        for k, part in pool.imap_unordered(_oracle_frame_k, list(enumerate(tasks)), chunksize=1):
            parts[k] = part
            _progress("oracle frame %d of %d done (%.1f s)" % (sum(p is not None for p in parts), len(tasks),
                                                               part[2]))
    except BaseException:
        pool.terminate()
        raise
    pool.close()
    pool.join()
    _progress("oracle workers joined")
    n_f = len(cfg["freqs"])
    evals = sum(n_rx * (bo[f + 1] - bo[f]) for f in frames) * n_f
    field_s = sum(p[2] for p in parts)
    occ_s = sum(p[3] for p in parts)
    timed_wall = max(p[2] for p in parts)
    E = d["out"].cpu().numpy()
    num, den = np.zeros(n_f), np.zeros(n_f)
    differ = 0
    for (f, idx), (E_own, E_frz, _, _) in zip(picks, parts):
        n = ro[f + 1] - ro[f]
        Eg = E[3 * n_f * ro[f]: 3 * n_f * ro[f + 1]].reshape(n_f, 3, n)[:, :, idx].astype(np.complex128)
        num += np.sum(np.abs(Eg - E_frz) ** 2, axis=(1, 2))
        den += np.sum(np.abs(E_frz) ** 2, axis=(1, 2))
        differ += int(np.sum(np.any(np.abs(E_own - E_frz) > 0, axis=(0, 1))))
    return {"value": evals / timed_wall, "unit": "evals/s", "cores": procs, "kind": "oracle",
            "sample": "%d crowd frames (seeded) x %d receivers each x their cylinders x %d frequencies = %d evals, "
                      "one process per frame; the slowest frame took %.1f s" % (len(frames), n_rx, n_f, evals,
                                                                               timed_wall),
            "occlusion_share_of_oracle_time": occ_s / field_s if field_s > 0 else None,
            "host": _host_info(),
            "fp32_field_error": {"max_normwise_rel": float(np.max(np.sqrt(num / den))),
                                 "receivers": n_rx * len(frames),
                                 "against": "FP64 oracle with the library's decisions, same float32 inputs",
                                 "receivers_whose_oracle_decisions_differ": differ}}


# ---------------------------------------------------------------------------

def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path (got --gpus %d); "
              "see the design notes for how the path would shard" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.copy_calibration_mib:
        a = torch.empty(args.copy_calibration_mib << 18, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    res = {"metric": "diffracted (rx*body*freq) evals/sec", "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic"}
    crowd = None
    if args.workload == "crowd":
        crowd = crowd_setup()
        _progress("crowd set up")
        ms, wall, k_ms, per_kernel, tune = crowd_batched(crowd, args.steps, args.warmup)
        _progress("crowd timed: %.3f ms per step" % ms)
        census = crowd_census(crowd)
        _progress("crowd path census done")
        cfg = crowd["cfg"]
        n_live = int(cfg["rx"].shape[0]) - census["inside"]
        field_flops = _path_flops(census, len(cfg["freqs"]), n_live)
        pairs = crowd["evals"] // len(cfg["freqs"])
        geom_flops = pairs * 3 * FLOPS_PATH_GEOM          # l_enc = 0: two creeping paths and the reflection
        flops = geom_flops + field_flops
        res.update({"value": crowd["evals"] / (ms / 1e3), "ms_per_step": ms, "wall_s": wall,
                    "config": {"workload": cfg["name"], "frames": len(cfg["body_off"]) - 1,
                               "receivers": int(cfg["rx"].shape[0]), "cylinders": int(cfg["cylinders"].shape[0]),
                               "frequencies": len(cfg["freqs"]), "triangles": int(cfg["tri"].shape[0]),
                               "evals_per_step": crowd["evals"], "tile": list(tune["best"]),
                               "parallelism": "single-gpu"},
                    "roofline": _alu_roofline(flops, k_ms, "k_batch<float,%d>" % tune["best"][0],
                                              {"traffic": measured_traffic("crowd", "utd::k_batch<float"),
                                               "paths": census["creeping"] + census["reflections"],
                                               "creeping": census["creeping"], "reflections": census["reflections"],
                                               "los_receivers": census["los"],
                                               "pairs": pairs, "geometry_flops": geom_flops,
                                               "field_flops": field_flops,
                                               "field_only_achieved": field_flops / (k_ms / 1e3) / 1e12,
                                               "note": "fused kernel (classification, reflection points, "
                                                       "visibility, field): 120 flops per candidate path "
                                                       "(3 per receiver-body pair) plus the field of the "
                                                       "visible paths"}),
                    "kernels_ms_per_step": per_kernel,
                    "tiles_ms": {"%dx%d" % k: v for k, v in tune["ms"].items()}})
    else:
        m = field_measure(args.workload, args.steps, args.warmup)
        res.update({"value": m["evals_per_s"], "ms_per_step": m["ms_per_step"],
                    "config": {"workload": m["workload"], "evals_per_step": m["evals_per_step"],
                               "parallelism": "single-gpu"},
                    "roofline": m["roofline"], "kernels_ms_per_step": m["kernels_ms_per_step"],
                    "visibility": m["visibility"]})
    if args.secondary:
        if crowd is not None:
            p_ms = crowd_per_frame(crowd, 2)
            res["per_frame"] = {"ms_per_step": p_ms, "evals_per_s": crowd["evals"] / (p_ms / 1e3),
                                "batched_over_per_frame_speedup": p_ms / res["ms_per_step"]}
            _progress("per-frame crowd timed")
        if args.workload != "sphere_plane":
            res["field"] = field_measure("sphere_plane", args.secondary_steps, 20)
            _progress("field workload timed")
        if args.workload != "room":
            res["occlusion"] = field_measure("room", max(10, args.secondary_steps // 10), 3)
            _progress("occlusion workload timed")
        res["adjoint"] = adjoint_measure(5)
        _progress("adjoint timed")
        res["caustic"] = caustic_measure(max(10, args.secondary_steps // 4), 3)
        _progress("caustic workload timed")
    if args.cpu_baseline and crowd is not None:
        _progress("CPU baseline (the oracle) starting")
        res["cpu_baseline"] = cpu_baseline(crowd, args.cpu_frames, args.cpu_rx)
        _progress("CPU baseline done")
    if crowd is not None:
        crowd["scene"].close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()

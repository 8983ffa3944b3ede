"""Throughput of the smooth-surface UTD field evaluation on one MI355X.

A step is one call of utd_smooth_field over the whole workload: per-body
constants, path classification and visibility (BVH + body tests), and the
coherent field of Eqs. (1)-(4) for every (receiver, body, frequency).
Default workload: PEC sphere a = 1 m, source at 4 m, 256 x 256 receivers on
the plane x = -3 m, 64 frequencies in 1-6 GHz, FP32 field with FP64 phase.
Inputs are resident in HBM before the timed region.

Prints one JSON line (rank 0).  ``--gpus`` above 1 is refused: this library
runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 operations per (path, frequency) of the field kernel, counted from its
# formula set for a creeping path (utd_fock.h / add_path): argument scaling 5,
# transition function 23 (index map 3, degree-4 complex Horner 16, combine
# into W = A0 + A1 v 4), regime lookup 42 (index map 2, degree-4 soft+hard
# complex Horner 32, combine 8), phase 30 (range reduction and degree-9/8
# sin/cos polynomials), phase times coefficients 12, accumulation into 3
# complex components 24.  The per-frequency k^{-1/6} scaling of each
# receiver's sum is not counted.  Direct field per (receiver, frequency): 36
# (phase 30 + 6 FMA).
FLOPS_PER_PATH_FREQ = 5 + 23 + 42 + 30 + 12 + 24
FLOPS_LOS = 36
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published, packed-FP32 rate)


TRAFFIC_PROFILE = {"config2": "profiles/hbm_sphere-plane-64f.md",
                   "config3": "profiles/hbm_room-512x512-2f.md"}


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


VIS_KERNELS = ("utd::k_setup", "utd::k_cand<float", "utd::k_vis<float", "utd::k_rec<float", "utd::k_paths<float")


def occlusion_summary(workload_name, prof, n_rx, n_body, n_paths, census):
    """Classification and visibility pass per call: time, active paths per
    (receiver, body) pair, and HBM bytes and GB/s from the committed PMC
    summary of the same kernels (null when it does not match the sources)."""
    occ_ms, occ_n = prof.get("occlude", (0.0, 0))
    ms = occ_ms / max(occ_n, 1)
    nbytes = None
    vals = [measured_traffic(workload_name, k) for k in VIS_KERNELS]
    if any(v is not None for v in vals):
        nbytes = sum(v for v in vals if v is not None)
    return {"ms": ms, "pairs": n_rx * max(n_body, 1), "active_paths": n_paths,
            "active_paths_per_pair": n_paths / max(n_rx * max(n_body, 1), 1),
            "los_receivers": census["los"], "hbm_bytes": nbytes,
            "hbm_GBps": (nbytes / (ms / 1e3) / 1e9) if (nbytes is not None and ms > 0) else None}


def measured_traffic(workload_name, kernel_prefix):
    """HBM bytes per launch of the field kernel from the committed PMC summary
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="config2", choices=["config2", "config3", "config5", "config1"])
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=1536, help="receivers in the oracle sample")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="also time forward + backward on the adjoint workload (room, 64 cylinders, 128^2 rx, 16 f)")
    ap.add_argument("--adjoint-steps", type=int, default=3)
    ap.add_argument("--batched", type=int, default=1,
                    help="also time the batched crowd workload (256 frames) against per-frame calls")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this size (HBM counter calibration under a profiler)")
    return ap.parse_args()


def workload(name):
    import workloads as W
    if name == "config2":
        return W.config2()
    if name == "config3":
        return W.config3()
    if name == "config5":
        return W.config5()
    return W.config1()


def cpu_baseline(cfg, n_sample, E_gpu=None):
    """The FP64 oracle on a bounded receiver sample, all frequencies, in a
    pool of worker processes (one receiver chunk each).  With the GPU field
    of the same call, also the error of that result on the sample (relative
    normwise per frequency, the largest over frequencies)."""
    import multiprocessing as mp

    import workloads as W
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(cfg["rx"].shape[0], n_sample, replace=False))
    sc, tx, rx = W.to_oracle(cfg["scene"], cfg["tx"], cfg["rx"][idx])
    cores = max(1, min(os.cpu_count() or 1, 16))
    chunks = np.array_split(np.arange(n_sample), cores)
    args = [(sc, tx, rx[c], cfg["freqs"]) for c in chunks if c.size]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(args)) as pool:
        parts = pool.map(_oracle_chunk, args)
    dt = time.perf_counter() - t0
    nb = len(sc["spheres"]) + len(sc["cylinders"])
    evals = n_sample * max(nb, 1) * len(cfg["freqs"])
    out = dict(value=evals / dt, unit="evals/s", cores=len(args), kind="oracle",
               sample="%d receivers x %d bodies x %d frequencies of the workload, %.1f s wall"
                      % (n_sample, nb, len(cfg["freqs"]), dt))
    if E_gpu is not None:
        Eo = np.concatenate(parts, axis=2)
        Eg = E_gpu[:, :, idx]
        num = np.sqrt(np.sum(np.abs(Eg - Eo) ** 2, axis=(1, 2)))
        den = np.sqrt(np.sum(np.abs(Eo) ** 2, axis=(1, 2)))
        out["fp32_field_error"] = {"max_normwise_rel": float(np.max(num / den)), "receivers": int(n_sample),
                                   "against": "FP64 oracle, same float32 inputs"}
    return out


def _oracle_chunk(a):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import field
    sc, tx, rx, freqs = a
    return field.field(sc, tx, rx, freqs)


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def adjoint_bench(steps):
    """Forward and backward (loss = sum |E|^2, so dL/dE = 2E) on the adjoint
    workload, FP32, inputs resident; the backward recomputes classification
    and visibility itself (it takes no state from the forward call)."""
    import torch

    import paper_2310_10578_amd as utd
    import workloads as W
    cfg = W.config5()
    dev = "cuda:0"
    sc = cfg["scene"]
    scene = utd.Scene(sc.get("tri"))
    sph = torch.from_numpy(np.ascontiguousarray(sc["spheres"], np.float32)).to(dev)
    cyl = torch.from_numpy(np.ascontiguousarray(sc["cylinders"], np.float32)).to(dev)
    rx = torch.from_numpy(cfg["rx"]).to(dev)
    freqs = torch.tensor(cfg["freqs"], dtype=torch.float64, device=dev)
    src = utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"])
    n_rx, n_f, n_body = rx.shape[0], freqs.shape[0], sph.shape[0] + cyl.shape[0]
    out = torch.empty((n_f, 3, n_rx), dtype=torch.complex64, device=dev)
    flags = torch.empty((n_rx,), dtype=torch.uint8, device=dev)
    utd.smooth_field(scene, sph, cyl, src, rx, freqs, out=out, flags=flags)
    gE = 2 * out
    fwd = _timed(lambda: utd.smooth_field(scene, sph, cyl, src, rx, freqs, out=out, flags=flags), steps, 1)
    bwd = _timed(lambda: utd.smooth_field_backward(scene, sph, cyl, src, rx, freqs, gE), steps, 1)
    utd.profile_enable(True)
    utd.profile_read()
    _timed(lambda: utd.smooth_field_backward(scene, sph, cyl, src, rx, freqs, gE), steps, 0)
    prof = utd.profile_read()
    utd.profile_enable(False)
    evals = n_rx * n_body * n_f
    scene.close()
    return {"workload": cfg["name"], "evals_per_step": evals, "fwd_ms": fwd, "bwd_ms": bwd,
            "bwd_over_fwd": bwd / fwd, "fwd_evals_per_s": evals / (fwd / 1e3),
            "bwd_evals_per_s": evals / (bwd / 1e3), "gradients": 3 + 3 * n_body,
            "bwd_kernels_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}}


def batched_bench(steps):
    """The crowd workload (256 frames of the room, 0-64 moving cylinders and
    1k-64k receivers per frame, 8 frequencies): one batched call (autotuned
    tiles, graph replay) against the same frames as per-frame calls."""
    import torch

    import paper_2310_10578_amd as utd
    import workloads as W
    from paper_2310_10578_amd.autotune import tune_batched
    cfg = W.config4()
    dev = "cuda:0"
    scene = utd.Scene(cfg["tri"])
    bo_h, ro_h = cfg["body_off"], cfg["rx_off"]
    bo = torch.from_numpy(bo_h).to(dev)
    ro = torch.from_numpy(ro_h).to(dev)
    cyl = torch.from_numpy(cfg["cylinders"]).to(dev)
    rx = torch.from_numpy(cfg["rx"]).to(dev)
    freqs = torch.tensor(cfg["freqs"], dtype=torch.float64, device=dev)
    src = utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"])
    n_rx, n_f = rx.shape[0], freqs.shape[0]
    out = torch.empty((3 * n_f * n_rx,), dtype=torch.complex64, device=dev)
    flags = torch.empty((n_rx,), dtype=torch.uint8, device=dev)
    tune = tune_batched(scene, bo, cyl, ro, rx, src, freqs, out=out, flags=flags)
    b_ms = _timed(lambda: utd.smooth_field_batched(scene, bo, cyl, ro, rx, src, freqs, out=out, flags=flags),
                  steps, 1)
    frames = []
    for f in range(len(bo_h) - 1):
        n = int(ro_h[f + 1] - ro_h[f])
        if n == 0:
            continue
        frames.append((cyl[bo_h[f]:bo_h[f + 1]], rx[ro_h[f]:ro_h[f + 1]],
                       out[3 * n_f * ro_h[f]: 3 * n_f * ro_h[f + 1]].view(n_f, 3, n), flags[ro_h[f]:ro_h[f + 1]]))

    def per_frame():
        for c, r, o, fl in frames:
            utd.smooth_field(scene, None, c, src, r, freqs, out=o, flags=fl)

    p_ms = _timed(per_frame, max(1, steps - 1), 1)
    nb = np.diff(bo_h)
    nr = np.diff(ro_h)
    evals = int((nb * nr).sum()) * n_f
    scene.close()
    return {"workload": cfg["name"], "frames": len(bo_h) - 1, "receivers": n_rx, "triangles": int(cfg["tri"].shape[0]),
            "evals_per_step": evals, "batched_ms": b_ms, "per_frame_ms": p_ms,
            "batched_evals_per_s": evals / (b_ms / 1e3), "per_frame_evals_per_s": evals / (p_ms / 1e3),
            "batched_over_per_frame_speedup": p_ms / b_ms,
            "tiles": {"best": list(tune["best"]), "ms": {"%dx%d" % k: v for k, v in tune["ms"].items()}}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU (this library has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2310_10578_amd as utd
    cfg = workload(args.workload)
    dev = "cuda:0"
    sc = cfg["scene"]
    scene = utd.Scene(sc.get("tri"))
    sph = torch.from_numpy(np.ascontiguousarray(sc["spheres"], np.float32)).to(dev)
    cyl = torch.from_numpy(np.ascontiguousarray(sc["cylinders"], np.float32)).to(dev)
    rx = torch.from_numpy(cfg["rx"]).to(dev)
    freqs = torch.tensor(cfg["freqs"], dtype=torch.float64, device=dev)
    src = utd.make_source(cfg["tx"]["pos"], cfg["tx"]["dipole"], cfg["tx"]["amplitude"])
    n_rx, n_f = rx.shape[0], freqs.shape[0]
    n_body = sph.shape[0] + cyl.shape[0]
    out = torch.empty((n_f, 3, n_rx), dtype=torch.complex64, device=dev)
    flags = torch.empty((n_rx,), dtype=torch.uint8, device=dev)

    def step():
        utd.smooth_field(scene, sph, cyl, src, rx, freqs, precision=0, out=out, flags=flags)

    if args.copy_calibration_mib:
        a = torch.empty(args.copy_calibration_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    # per-kernel durations: the same steps again with the library's event
    # hook (HIP events around each launch, on the launch stream); kept out
    # of the timed loop above so the markers do not stretch the step
    utd.profile_enable(True)
    utd.profile_read()
    for _ in range(args.steps):
        step()
    prof = utd.profile_read()
    utd.profile_enable(False)

    # algorithmic work of the field kernel: the paths it evaluates, from the
    # library's path census of the same inputs (outside the timed region)
    census = utd.path_census(scene, sph, cyl, src, rx)
    n_paths, los = census["paths"], census["los"]
    flops = (n_paths * FLOPS_PER_PATH_FREQ + los * FLOPS_LOS) * n_f
    field_ms, field_n = prof["field"]
    field_avg_s = field_ms / max(field_n, 1) / 1e3
    achieved = flops / field_avg_s / 1e12
    ms_step = ms_total / args.steps
    evals = n_rx * max(n_body, 1) * n_f
    res = {
        "metric": "diffracted (rx*body*freq) evals/sec",
        "value": evals / (ms_step / 1e3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "receivers": n_rx, "bodies": n_body, "frequencies": n_f,
                   "triangles": scene.n_tri, "evals_per_step": evals, "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(args.workload, "utd::k_field<float"),
                     "kernel": "k_field<float>", "kernel_ms": field_avg_s * 1e3,
                     "flops_per_launch": flops, "paths": n_paths, "los_receivers": los},
        "kernels_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]},
        "occlusion": occlusion_summary(args.workload, prof, n_rx, n_body, n_paths, census),
        "wall_s": wall,
    }
    if args.adjoint:
        res["adjoint"] = adjoint_bench(args.adjoint_steps)
    if args.batched:
        res["batched"] = batched_bench(args.batched_steps)
    if args.cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cfg, min(args.cpu_sample, n_rx), out.cpu().numpy().astype(np.complex128))
    print(json.dumps(res))




if __name__ == "__main__":
    main()

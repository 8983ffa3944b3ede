"""Helpers shared by the GPU tests: run the HIP library through its binding
and compare against the oracle on the same float32-rounded inputs."""
import numpy as np

import workloads as W


def run_library(cfg, precision=0, rx=None, freqs=None, **kw):
    import torch

    import paper_2310_10578_amd as utd
    sc = cfg["scene"]
    scene = utd.Scene(sc.get("tri"))
    sph = torch.from_numpy(np.ascontiguousarray(sc["spheres"], np.float32)).cuda()
    cyl = torch.from_numpy(np.ascontiguousarray(sc["cylinders"], np.float32)).cuda()
    rx = cfg["rx"] if rx is None else rx
    freqs = cfg["freqs"] if freqs is None else freqs
    rxt = torch.from_numpy(np.ascontiguousarray(rx, np.float32)).cuda()
    ft = torch.from_numpy(np.ascontiguousarray(freqs, np.float64)).cuda()
    tx = cfg["tx"]
    src = utd.make_source(tx["pos"], tx["dipole"], tx["amplitude"])
    E, flags = utd.smooth_field(scene, sph, cyl, src, rxt, ft, precision=precision, **kw)
    torch.cuda.synchronize()
    out = E.cpu().numpy().astype(np.complex128), flags.cpu().numpy()
    scene.close()
    return out


def run_oracle(cfg, rx=None, freqs=None, opts=None):
    from oracle import field
    sc, tx, r = W.to_oracle(cfg["scene"], cfg["tx"], cfg["rx"] if rx is None else rx)
    freqs = cfg["freqs"] if freqs is None else freqs
    E, info = field.field(sc, tx, r, freqs, opts=opts, return_info=True)
    return E, info


def normwise(Eg, Eo):
    """Per frequency ||E_gpu - E_ref||_2 / ||E_ref||_2 over all receivers and components."""
    num = np.sqrt(np.sum(np.abs(Eg - Eo) ** 2, axis=(1, 2)))
    den = np.sqrt(np.sum(np.abs(Eo) ** 2, axis=(1, 2)))
    return num / den

"""Gradients of a real loss of the oracle field, FP64, by finite differences.

Test infrastructure (see ``oracle/__init__``).

For a complex weight G[f, c, n] the loss is L(theta) = Re sum conj(G) E(theta)
(so dL/dE = G in PyTorch's complex convention).  The field of Eqs. (1)-(4)
is a smooth function of the source position and of every body's centre and
radius as long as no path changes visibility or existence; the derivative
is taken there, with the classification of the unperturbed inputs frozen
(``field(..., frozen=...)``), by central differences
    D(h) = (L(theta + h e) - L(theta - h e)) / (2 h)
extrapolated once (Richardson): (4 D(h/2) - D(h)) / 3, whose error is
O(h^4) in the field's fourth derivative (for a phase e^{-jks} about
(k h)^4 / 480 relative).

Parameters: the source position (3), per sphere (cx, cy, cz, a), per
cylinder (cx, cy, a); cylinder heights only move visibility boundaries.
"""
import copy

import numpy as np

from . import field as F


def loss(E, G):
    return float(np.sum((np.conj(G) * E).real))


def _params(scene):
    """(group, index, column) of every differentiable parameter."""
    out = [("tx", 0, c) for c in range(3)]
    sph = np.asarray(scene.get("spheres", np.zeros((0, 4))), float).reshape(-1, 4)
    cyl = np.asarray(scene.get("cylinders", np.zeros((0, 5))), float).reshape(-1, 5)
    out += [("sph", i, c) for i in range(sph.shape[0]) for c in range(4)]
    out += [("cyl", i, c) for i in range(cyl.shape[0]) for c in (0, 1, 4)]
    return out


def _perturbed(scene, tx, p, delta):
    sc = {k: (np.array(v, dtype=float, copy=True) if v is not None else None) for k, v in scene.items()}
    t = copy.deepcopy(tx)
    t["pos"] = np.array(tx["pos"], dtype=float, copy=True)
    group, i, c = p
    if group == "tx":
        t["pos"][c] += delta
    elif group == "sph":
        sc["spheres"] = sc["spheres"].reshape(-1, 4)
        sc["spheres"][i, c] += delta
    else:
        sc["cylinders"] = sc["cylinders"].reshape(-1, 5)
        sc["cylinders"][i, c] += delta
    return sc, t


def loss_grad(scene, tx, rx, freqs, G, opts=None, h=1e-5, bodies=None):
    """dL/dtheta for every parameter: dict(tx [3], sph [ns, 4], cyl [nc, 3]).

    ``h`` is the largest step (metres); the frozen classification is that of
    the unperturbed inputs.  ``bodies``: optional list of ("sph", i) /
    ("cyl", i) whose parameters are differentiated (the others stay 0);
    default all."""
    scene = dict(scene)
    scene.setdefault("spheres", np.zeros((0, 4)))
    scene.setdefault("cylinders", np.zeros((0, 5)))
    E0, info = F.field(scene, tx, rx, freqs, opts=opts, return_info=True)

    def L(p, delta):
        sc, t = _perturbed(scene, tx, p, delta)
        return loss(F.field(sc, t, rx, freqs, opts=opts, frozen=info), G)

    ns = np.asarray(scene["spheres"]).reshape(-1, 4).shape[0]
    nc = np.asarray(scene["cylinders"]).reshape(-1, 5).shape[0]
    out = dict(tx=np.zeros(3), sph=np.zeros((ns, 4)), cyl=np.zeros((nc, 3)))
    for p in _params(scene):
        if bodies is not None and p[0] != "tx" and (p[0], p[1]) not in bodies:
            continue
        d1 = (L(p, h) - L(p, -h)) / (2 * h)
        d2 = (L(p, h / 2) - L(p, -h / 2)) / h
        d = (4 * d2 - d1) / 3
        group, i, c = p
        if group == "tx":
            out["tx"][c] = d
        elif group == "sph":
            out["sph"][i, c] = d
        else:
            out["cyl"][i, {0: 0, 1: 1, 4: 2}[c]] = d
    return out


def flatten(g):
    return np.concatenate([np.ravel(g["tx"]), np.ravel(g["sph"]), np.ravel(g["cyl"])])

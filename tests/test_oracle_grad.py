"""Pins of the oracle's loss gradient (finite differences with the
classification frozen): a closed-form derivative of the direct ray, the
translation invariance of a scene without occluding triangles, the
electrical scaling law (which exercises the radius derivatives) and the
step-size convergence of the extrapolated differences."""
import numpy as np
import pytest

from oracle import field as F
from oracle import grad

C0 = 299792458.0


def _weights(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _scene_mixed():
    return dict(spheres=np.array([[0.2, -0.3, 1.1, 0.35], [-1.6, 0.9, 0.8, 0.25]]),
                cylinders=np.array([[1.4, 0.8, 0.0, 2.5, 0.3], [-0.4, 1.9, 0.0, 2.5, 0.2]]))


def _receivers(n, seed, r=(2.5, 4.0)):
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, n)
    rr = rng.uniform(*r, n)
    return np.stack([rr * np.cos(ph), rr * np.sin(ph), rng.uniform(0.4, 1.6, n)], 1)


TX = dict(pos=np.array([3.1, -0.7, 1.2]), dipole=np.array([0.3, -0.2, 1.0]), amplitude=1.7)


def test_direct_ray_gradient_closed_form():
    """No bodies: dL/dT of the dipole's ray field against its analytic
    derivative (s = |R - T|, s-hat = (R - T)/s,
    E = A (p - (p.s-hat) s-hat) e^{-jks}/s)."""
    R = _receivers(40, 1)
    freqs = np.array([2e9, 9e9])
    G = _weights((2, 3, 40), 2)
    g = grad.loss_grad(dict(), TX, R, freqs, G)
    p, A, T = TX["dipole"], TX["amplitude"], TX["pos"]
    want = np.zeros(3)
    for fi, f in enumerate(freqs):
        k = 2 * np.pi * f / C0
        for n in range(R.shape[0]):
            v = R[n] - T
            s = np.linalg.norm(v)
            sh = v / s
            w = p - (p @ sh) * sh
            phi = np.exp(-1j * k * s) / s
            dphi = (-1j * k - 1 / s) * phi
            for j in range(3):
                dsh = (np.eye(3)[j] - sh * sh[j]) / s          # d s-hat / d v_j
                dw = -((p @ dsh) * sh + (p @ sh) * dsh)
                dE_dv = A * (dw * phi + w * dphi * sh[j])
                want[j] -= np.sum((np.conj(G[fi, :, n]) * dE_dv).real)   # dv/dT = -1
    np.testing.assert_allclose(g["tx"], want, rtol=1e-8)


def _frozen_loss(scene, tx, R, freqs, G, info):
    return grad.loss(F.field(scene, tx, R, freqs, frozen=info), G)


def _richardson(fun, h):
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(h / 2) - fun(-h / 2)) / h
    return (4 * d2 - d1) / 3


def test_translation_invariance():
    """Without triangles, moving the source and every body by d equals moving
    every receiver by -d, so the centre and source gradients sum to minus the
    derivative of L under a common receiver shift (per axis)."""
    sc = _scene_mixed()
    R = _receivers(48, 3)
    freqs = np.array([3e9, 11e9])
    G = _weights((2, 3, 48), 4)
    g = grad.loss_grad(sc, TX, R, freqs, G)
    _, info = F.field(sc, TX, R, freqs, return_info=True)
    for ax in range(3):
        e = np.eye(3)[ax]
        dR = _richardson(lambda d: _frozen_loss(sc, TX, R + d * e, freqs, G, info), 1e-5)
        tot = g["tx"][ax] + g["sph"][:, ax].sum() + (g["cyl"][:, ax].sum() if ax < 2 else 0.0)
        assert abs(tot + dR) <= 1e-7 * (abs(dR) + np.abs(g["tx"]).max())


def test_electrical_scaling_law():
    """Scaling every length by alpha and the frequency by 1/alpha scales the
    field by 1/alpha (all Fock and transition arguments are invariant), so
    sum_theta theta dL/dtheta (source, centres, radii, receivers) - f dL/df = -L.
    The radius terms make this a pin of the radius derivatives."""
    sc = _scene_mixed()
    R = _receivers(48, 5)
    freqs = np.array([4e9])
    G = _weights((1, 3, 48), 6)
    g = grad.loss_grad(sc, TX, R, freqs, G)
    E0, info = F.field(sc, TX, R, freqs, return_info=True)
    L0 = grad.loss(E0, G)
    dR = _richardson(lambda d: _frozen_loss(sc, TX, R * (1 + d), freqs, G, info), 1e-6)
    df = _richardson(lambda d: _frozen_loss(sc, TX, R, freqs * (1 + d), G, info), 1e-6)
    s = TX["pos"] @ g["tx"]
    s += np.sum(sc["spheres"] * g["sph"])
    s += np.sum(sc["cylinders"][:, [0, 1, 4]] * g["cyl"])
    lhs = s + dR - df
    assert abs(lhs + L0) <= 1e-6 * (abs(s) + abs(dR) + abs(df))


def test_extrapolated_differences_converge():
    """Halving and quadrupling the step changes the gradient by far less than
    the tolerances the GPU adjoint is held to."""
    sc = _scene_mixed()
    R = _receivers(32, 7)
    freqs = np.array([28e9])
    G = _weights((1, 3, 32), 8)
    a = grad.flatten(grad.loss_grad(sc, TX, R, freqs, G, h=1e-5))
    b = grad.flatten(grad.loss_grad(sc, TX, R, freqs, G, h=4e-5))
    assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(a)


@pytest.mark.parametrize("shift", [1e-3])
def test_frozen_gradient_matches_unfrozen_difference_away_from_boundaries(shift):
    """Where no receiver is near a visibility boundary, freezing the
    classification changes nothing: a plain central difference of the
    unfrozen oracle at a step that flips no decision agrees with the frozen
    gradient to the step's O(h^2) error."""
    sc = dict(spheres=np.array([[0.0, 0.0, 1.0, 0.4]]))
    R = _receivers(24, 9, r=(2.5, 3.0))
    R[:, 2] = 1.0
    freqs = np.array([1e9])
    G = _weights((1, 3, 24), 10)
    g = grad.loss_grad(sc, TX, R, freqs, G)
    sp = dict(spheres=sc["spheres"] + np.array([[0, 0, 0, shift]]))
    sm = dict(spheres=sc["spheres"] - np.array([[0, 0, 0, shift]]))
    _, ip = F.field(sp, TX, R, freqs, return_info=True)
    _, im = F.field(sm, TX, R, freqs, return_info=True)
    _, i0 = F.field(sc, TX, R, freqs, return_info=True)
    same = all(np.array_equal(a[1]["valid"], b[1]["valid"]) and np.array_equal(a[1]["valid"], c[1]["valid"])
               for a, b, c in zip(i0["paths"], ip["paths"], im["paths"]))
    assert same
    d = (grad.loss(F.field(sp, TX, R, freqs), G) - grad.loss(F.field(sm, TX, R, freqs), G)) / (2 * shift)
    k = 2 * np.pi * freqs[0] / C0
    assert abs(d - g["sph"][0, 3]) <= 2 * (k * shift) ** 2 * abs(d) + 1e-12

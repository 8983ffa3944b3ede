"""Pins of the oracle's uniform field at a sphere's axial caustic
(``caustic_uniform``): the exact series on and near the rear axis, the
two-ray limit far from it, reciprocity on the axis and continuity onto it."""
import numpy as np
import pytest

from oracle import caustic, field, mie

C0 = 299792458.0
A, B = 0.5, 3.0
OPT = dict(caustic_uniform=True)


def _near_axis(deg, r=3.0):
    th = np.radians(np.asarray(deg, dtype=float))
    return th, np.stack([r * np.cos(th), r * np.sin(th), np.zeros_like(th)], 1)


DEG = [175, 177, 178, 179, 179.5, 179.9, 180.0]


@pytest.mark.parametrize("mode,bounds", [("soft", (2.45, 1.15, 0.8)), ("hard", (0.45, 0.45, 0.45))])
def test_scalar_uniform_field_vs_mie_on_the_rear_axis(mode, bounds):
    """Within 5 degrees of the rear axis (the axis itself included, where the
    ray field is infinite) the uniform field follows the exact series as
    closely as the ray field does elsewhere in the shadow, and the soft
    error falls with ka as the neglected O(m^-2) terms do."""
    th, rx = _near_axis(DEG)
    worst = []
    for f, bound in zip((1e9, 3e9, 6e9), bounds):
        k = 2 * np.pi * f / C0
        u = field.field(dict(spheres=[[0, 0, 0, A]]), dict(pos=[B, 0, 0]), rx, [f], mode=mode, opts=OPT)[0]
        ue = mie.sphere_scalar(k, A, B, np.full(th.size, 3.0), th, hard=(mode == "hard"))
        dB = 20 * np.log10(np.abs(u) / np.abs(ue))
        assert np.all(np.isfinite(dB)) and np.max(np.abs(dB)) < bound
        worst.append(np.max(np.abs(dB)))
    if mode == "soft":
        np.testing.assert_allclose([worst[0] / worst[1], worst[1] / worst[2]], [3 ** (2 / 3), 2 ** (2 / 3)],
                                   rtol=0.3)


def test_em_uniform_field_vs_mie_radial_dipole_on_the_rear_axis():
    """Radial dipole (the hard polarisation with the axial terms) against the
    exact Debye series on and near the rear axis; the error falls with ka."""
    th, rx = _near_axis(DEG)
    worst = []
    for f, bound in zip((1e9, 3e9, 6e9), (2.9, 1.2, 0.8)):
        k = 2 * np.pi * f / C0
        E = field.field(dict(spheres=[[0, 0, 0, A]]), dict(pos=[B, 0, 0], dipole=[1.0, 0, 0]), rx, [f], opts=OPT)[0]
        Mr, Mt = mie.sphere_radial_dipole(k, A, B, np.stack([np.full(th.size, 3.0), th], 1))
        dB = 20 * np.log10(np.linalg.norm(np.abs(E), axis=0) / (np.sqrt(np.abs(Mr) ** 2 + np.abs(Mt) ** 2) / k ** 2))
        assert np.max(np.abs(dB)) < bound
        worst.append(np.max(np.abs(dB)))
    np.testing.assert_allclose([worst[0] / worst[1], worst[1] / worst[2]], [3 ** (2 / 3), 2 ** (2 / 3)], rtol=0.4)


@pytest.mark.parametrize("l_enc", [0, 1, 2])
def test_uniform_field_tends_to_the_two_rays(l_enc):
    """Away from the axis each pair's uniform field is the sum of its two
    rays up to the O(1/x) of the Bessel functions' asymptotic forms
    (x = k a eps), measured against the pair's own ray magnitudes: a swapped
    Bessel combination, a lost phase or quarter turn or a wrong amplitude
    would leave an O(1) difference.  Rear pairs on both sides of
    theta_R + gamma_R = pi (the far ray's extra caustic on the surface or in
    space), front pairs from l_enc 1; a tilted dipole exercises every
    polarisation term; receivers off the source plane."""
    th = np.radians(np.concatenate([np.linspace(92, 172, 24), np.linspace(8, 88, 12)]))
    rx = np.stack([2.5 * np.cos(th), 2.5 * np.sin(th) * 0.6, 2.5 * np.sin(th) * 0.8], 1)
    T, dip = np.array([B, 0, 0]), np.array([0.3, 0.5, 0.8])
    sc = dict(spheres=[[0, 0, 0, A]])
    info = field.classify(sc, T, rx, dict(OPT, l_enc=l_enc))
    assert sum(len(p[4]) for p in info["pairs"]) >= (4, 40, 76)[l_enc]
    for f in (5e9, 10e9, 20e9):
        k = 2 * np.pi * f / C0
        for C, a, near, far, idx, rear in info["pairs"]:
            Eu = np.zeros((3, rx.shape[0]), complex)
            caustic.add_pair(Eu, T, C, a, rx, near, far, idx, rear, dip, 1.0, k, "em")
            En, Ef = np.zeros_like(Eu), np.zeros_like(Eu)
            field._add_creeping(En, near, idx, T, dip, 1.0, k, "em")
            field._add_creeping(Ef, far, idx, T, dip, 1.0, k, "em")
            x = k * a * np.where(rear, np.pi - th[idx], th[idx])
            rel = np.linalg.norm(Eu - En - Ef, axis=0)[idx] / (np.linalg.norm(En, axis=0) + np.linalg.norm(Ef, axis=0))[idx]
            assert np.max(rel * x) < 3.0, (f, rear, np.max(rel * x))


def info_pairs(sc, tx, rx, l_enc):
    return field.classify(sc, tx["pos"], rx, dict(OPT, l_enc=l_enc))["pairs"]


def test_uniform_field_on_the_axis():
    """On the axis the field is finite, the receiver is not flagged, the
    field is reciprocal (q.E_p(R) = p.E_q(T)), and the axis is reached
    continuously from every side."""
    sc = dict(spheres=[[0.1, -0.2, 0.05, A]])
    T = np.array([3.0, 0.4, -0.3])
    C = np.array(sc["spheres"][0][:3])
    ax = (C - T) / np.linalg.norm(C - T)
    R = C + 2.2 * ax
    p, q = np.array([0.3, -0.7, 0.2]), np.array([0.5, 0.1, -0.4])
    e1 = np.cross(ax, [0, 0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(ax, e1)
    for l_enc in (0, 1):
        for f in (1e9, 3.5e9):
            o = dict(OPT, l_enc=l_enc)
            Ep, info = field.field(sc, dict(pos=T, dipole=p), R[None], [f], opts=o, return_info=True)
            Eq = field.field(sc, dict(pos=R, dipole=q), T[None], [f], opts=o)
            assert info["flags"][0] & field.FLAG_CAUSTIC == 0 and np.all(np.isfinite(Ep))
            lhs, rhs = q @ Ep[0][:, 0], p @ Eq[0][:, 0]
            assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
            near = R + 1e-7 * np.stack([e1, e2, -e1, -e2, (e1 + e2) / np.sqrt(2)])
            En = field.field(sc, dict(pos=T, dipole=p), near, [f], opts=o)[0]
            assert np.max(np.abs(En - Ep[0][:, :1])) <= 1e-5 * np.max(np.abs(Ep))
    # without the option the axis keeps its flag and drops the paths
    E0, info = field.field(sc, dict(pos=T, dipole=p), R[None], [1e9], return_info=True)
    assert info["flags"][0] & field.FLAG_CAUSTIC


def test_sphere_frame_on_the_axis_is_orthonormal():
    """On the axis the plane of the path is any plane through it: the frame
    must still be orthonormal (normalising rounding noise would not be)."""
    from oracle import geometry
    T = np.array([3.0, 0.4, -0.3])
    C = np.array([0.1, -0.2, 0.05])
    ax = (C - T) / np.linalg.norm(C - T)
    R = (C + 2.2 * ax)[None]
    dT, eT, dR, ep, thR = geometry.sphere_frame(T, C, A, R)
    assert abs(ep[0] @ eT) < 1e-15 and abs(np.linalg.norm(ep[0]) - 1) < 1e-15
    rec = geometry.sphere_creeping(T, C, A, R, +1, 0)
    assert abs(np.linalg.norm(rec["n2"][0]) - 1) < 1e-14 and abs(rec["n1"][0] @ rec["b1"][0]) < 1e-14

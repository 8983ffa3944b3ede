"""Pins of the oracle's wall bounces (one specular reflection on the scene's
planes, alone and feeding the bodies) against what the physics fixes:

* a perfectly conducting plane: the reflected ray field is exactly the ray
  field of the image dipole -p + 2 (p.n) n at the image point;
* the slab coefficients: energy balance |R|^2 + |T|^2 = 1 of a lossless slab,
  the Brewster angle of a lossless half-space, R_perp = -R_par at normal
  incidence, a thick lossy slab tends to the half-space, a very lossy one to
  the perfect conductor;
* a wall-then-body creeping path off a perfectly conducting wall equals the
  creeping path of the image source with the image dipole (the wall's
  polarisation mapping and the equivalent-source geometry);
* reciprocity of the whole field with brick walls and bodies.
"""
import numpy as np
import pytest

from oracle import field, walls

F0 = 5e9


def _plane_tris(z=0.0, half=50.0):
    """A large square in the plane z = const, two triangles."""
    a, b, c, d = (-half, -half, z), (half, -half, z), (half, half, z), (-half, half, z)
    return np.array([[a, b, c], [a, c, d]], float)


def test_pec_plane_is_the_image_dipole():
    rng = np.random.default_rng(1)
    T = np.array([0.3, -0.2, 1.7])
    p = np.array([0.4, -0.7, 0.55])
    R = np.stack([rng.uniform(-4, 4, 64), rng.uniform(-4, 4, 64), rng.uniform(0.2, 3.0, 64)], 1)
    sc = dict(tri=_plane_tris())
    E_all, info = field.field(sc, dict(pos=T, dipole=p, amplitude=1.3), R, [F0],
                              opts=dict(walls=walls.PEC), return_info=True)
    E_dir = field.field(dict(tri=None), dict(pos=T, dipole=p, amplitude=1.3), R, [F0])
    assert all(rec["valid"].all() for key, rec in info["walls"] if key[0] == "w")
    # image: T' = (x, y, -z), dipole -p + 2 (p.n) n
    n = np.array([0.0, 0.0, 1.0])
    Ti = T * np.array([1, 1, -1.0])
    pi = -p + 2 * (p @ n) * n
    E_img = field.field(dict(tri=None), dict(pos=Ti, dipole=pi, amplitude=1.3), R, [F0])
    np.testing.assert_allclose(E_all - E_dir, E_img, rtol=0, atol=1e-13 * np.abs(E_img).max())


@pytest.mark.parametrize("sigma", [0.0])
def test_lossless_slab_energy_balance(sigma):
    mat = dict(eps_r=3.75, sigma=sigma, thickness=0.1)
    cos_t = np.linspace(0.02, 1.0, 50)
    for f in (1e9, 2.4e9, 5e9, 28e9):
        Rp, Rl = walls.slab_coefficients(cos_t, f, mat)
        Tp, Tl = walls.slab_transmission(cos_t, f, mat)
        np.testing.assert_allclose(np.abs(Rp) ** 2 + np.abs(Tp) ** 2, 1.0, atol=1e-13)
        np.testing.assert_allclose(np.abs(Rl) ** 2 + np.abs(Tl) ** 2, 1.0, atol=1e-13)
        # a lossless slab reflects somewhere strictly between 0 and 1
        assert np.all(np.abs(Rp) < 1) and np.all(np.abs(Rp).max() > 0.1)


def test_half_space_brewster_and_normal_incidence():
    er = 3.75
    half = dict(eps_r=er, sigma=0.0, thickness=np.inf)
    th_b = np.arctan(np.sqrt(er))
    Rp, Rl = walls.slab_coefficients(np.array([np.cos(th_b)]), F0, half)
    assert abs(Rl[0]) < 1e-14 and abs(Rp[0]) > 0.3
    Rp, Rl = walls.slab_coefficients(np.array([1.0]), F0, half)
    np.testing.assert_allclose(Rp, -Rl, atol=1e-15)
    np.testing.assert_allclose(Rp, (1 - np.sqrt(er)) / (1 + np.sqrt(er)), atol=1e-15)
    # grazing incidence: both tend to -1 on a dielectric
    Rp, Rl = walls.slab_coefficients(np.array([1e-7]), F0, half)
    np.testing.assert_allclose([Rp[0], Rl[0]], [-1, -1], atol=1e-5)


def test_slab_limits():
    cos_t = np.linspace(0.05, 1.0, 20)
    # thick and lossy: the back face no longer matters
    thick = walls.slab_coefficients(cos_t, F0, dict(eps_r=3.75, sigma=2.0, thickness=5.0))
    half = walls.slab_coefficients(cos_t, F0, dict(eps_r=3.75, sigma=2.0, thickness=np.inf))
    np.testing.assert_allclose(thick[0], half[0], atol=1e-12)
    np.testing.assert_allclose(thick[1], half[1], atol=1e-12)
    # a good conductor is nearly the perfect conductor (R_perp -> -1, R_par -> +1)
    Rp, Rl = walls.slab_coefficients(cos_t, F0, dict(eps_r=1.0, sigma=1e9, thickness=0.1))
    np.testing.assert_allclose(Rp, -1, atol=2e-3)
    np.testing.assert_allclose(Rl, 1, atol=2e-3 / cos_t.min())
    # a thin slab (k t << 1) reflects to first order in k t:
    #   R_perp = j k t (1 - eta) / (2 cos),  R_par = j k t (eta^2 cos^2 - eta + sin^2) / (2 eta cos)
    t = 1e-8
    mat = dict(eps_r=3.75, sigma=0.038, thickness=t)
    Rp, Rl = walls.slab_coefficients(cos_t, F0, mat)
    k = 2 * np.pi * F0 / walls.C0
    eta = 3.75 - 1j * 0.038 / (2 * np.pi * F0 * walls.EPS0)
    sin2 = 1 - cos_t ** 2
    np.testing.assert_allclose(Rp, 1j * k * t * (1 - eta) / (2 * cos_t), rtol=1e-3)
    np.testing.assert_allclose(Rl, 1j * k * t * (eta ** 2 * cos_t ** 2 - eta + sin2) / (2 * eta * cos_t), rtol=1e-3)


@pytest.mark.parametrize("body", ["sphere", "cylinder"])
def test_wall_fed_creeping_is_the_image_source_path(body):
    """With a perfectly conducting wall (the plane x = 0), the wall-then-body
    creeping and reflected paths equal the paths of the image source with the
    image dipole, on every receiver where they are valid."""
    T = np.array([1.4, 0.5, 1.6])
    p = np.array([0.2, 0.6, 0.77])
    if body == "sphere":
        sc = dict(tri=None, spheres=np.array([[3.0, 2.5, 1.2, 0.4]]))
    else:
        sc = dict(tri=None, cylinders=np.array([[3.0, 2.5, 0.0, 3.0, 0.35]]))
    # receivers behind the body as seen from the wall's image of the source
    yy, zz = np.meshgrid(np.linspace(3.6, 6.0, 9), np.linspace(0.6, 1.8, 5), indexing="ij")
    R = np.stack([np.full(yy.size, 4.5), yy.ravel(), zz.ravel()], 1)
    wall = np.array([[[0, -20, -20], [0, 20, -20], [0, 20, 20]], [[0, -20, -20], [0, 20, 20], [0, -20, 20]]], float)
    sc_w = dict(sc, tri=wall)
    tx = dict(pos=T, dipole=p, amplitude=1.0)
    _, info = field.field(sc_w, tx, R, [F0], opts=dict(walls=walls.PEC), return_info=True)
    n = np.array([1.0, 0.0, 0.0])
    Ti = T * np.array([-1.0, 1, 1])
    pi = -p + 2 * (p @ n) * n
    tx_i = dict(pos=Ti, dipole=pi, amplitude=1.0)
    _, info_i = field.field(sc, tx_i, R, [F0], return_info=True)
    checked = 0
    for key, rec in info["walls"]:
        if key[0] != "wb":
            continue
        valid = rec["valid"]
        if not valid.any():
            continue
        # the same path of the image source, alone
        only = lambda recs, k: [(kk, dict(valid=(r["valid"] & valid) if kk == k else np.zeros_like(valid)))
                                for kk, r in recs]
        fz_w = dict(los=np.zeros(len(R), bool), inside=info["inside"], flags=info["flags"],
                    paths=only(info["paths"], None),
                    walls=[(kk, dict(valid=valid if kk == key else np.zeros_like(valid))) for kk, _ in info["walls"]])
        Ew = field.field(sc_w, tx, R, [F0], opts=dict(walls=walls.PEC), frozen=fz_w)
        bkey = key[2] + key[3]
        fz_i = dict(los=np.zeros(len(R), bool), inside=info_i["inside"], flags=info_i["flags"],
                    paths=only(info_i["paths"], bkey))
        Ei = field.field(sc, tx_i, R, [F0], frozen=fz_i)
        np.testing.assert_allclose(Ew, Ei, rtol=0, atol=1e-12 * np.abs(Ei).max())
        checked += int(valid.sum())
    assert checked >= 20


def test_reciprocity_with_brick_walls_and_bodies():
    """q.E_p(R) = p.E_q(T) for the whole field (direct ray, bodies, wall
    bounces alone and feeding the bodies in both orders) in a box of brick
    walls with a sphere and a cylinder."""
    rng = np.random.default_rng(7)
    L = (6.0, 5.0, 3.0)
    tri = []
    for ax in range(3):
        for side in (0.0, L[ax]):
            o = [0.0, 0.0, 0.0]
            o[ax] = side
            u = [0.0, 0.0, 0.0]
            v = [0.0, 0.0, 0.0]
            u[(ax + 1) % 3] = L[(ax + 1) % 3]
            v[(ax + 2) % 3] = L[(ax + 2) % 3]
            o, u, v = map(np.array, (o, u, v))
            tri += [[o, o + u, o + u + v], [o, o + u + v, o + v]]
    sc = dict(tri=np.array(tri), spheres=np.array([[2.2, 3.1, 1.0, 0.35]]),
              cylinders=np.array([[4.1, 1.6, 0.0, 1.7, 0.25]]))
    opts = dict(walls=walls.BRICK, l_enc=1)
    tested = 0
    for _ in range(6):
        T = rng.uniform([0.5, 0.5, 0.3], [5.5, 4.5, 2.7])
        R = rng.uniform([0.5, 0.5, 0.3], [5.5, 4.5, 2.7])
        if field.source_inside(sc, T) or field.source_inside(sc, R):
            continue
        p, q = rng.standard_normal(3), rng.standard_normal(3)
        Ep = field.field(sc, dict(pos=T, dipole=p), R[None, :], [2.4e9, 5e9], opts=opts)[:, :, 0]
        Eq = field.field(sc, dict(pos=R, dipole=q), T[None, :], [2.4e9, 5e9], opts=opts)[:, :, 0]
        np.testing.assert_allclose(Ep @ q, Eq @ p, rtol=1e-11)
        tested += 1
    assert tested >= 4

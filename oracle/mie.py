"""Exact eigenfunction series for PEC bodies (validation of the oracle only).

Test infrastructure (see ``oracle/__init__``).  The paper validates its sphere
fields against the analytic solution (Sec. IV-A, citing Jin); these are the
classical series, time factor e^{+jwt}, h_n = h_n^{(2)} (outgoing).

* ``sphere_scalar``: point source u^i = e^{-jkR}/R at distance b on the
  z-axis of a sphere of radius a with u = 0 (soft) or du/dn = 0 (hard):
      u^i = -jk sum (2n+1) j_n(k r<) h_n(k r>) P_n(cos th)
      u^s =  jk sum (2n+1) [j_n(ka)/h_n(ka) | j_n'(ka)/h_n'(ka)] h_n(kb) h_n(kr) P_n(cos th)
* ``sphere_radial_dipole``: electric dipole along the radius (z) at r = b,
  E = curl curl (z e^{-jkR}/R).  The field is TM to r; with the Debye
  potential u = sum u_n(r) P_n(cos th),
      E_r = sum n(n+1) u_n/r P_n,  E_th = sum (1/r) d(r u_n)/dr dP_n/dth,
      u_n^i = -jk (2n+1)/b j_n(k r<) h_n(k r>),
      u_n^s = +jk (2n+1)/b [J_n'(ka)/H_n'(ka)] h_n(kb) h_n(kr)
  with the Riccati functions J_n(x) = x j_n(x), H_n(x) = x h_n(x) (E_th = 0
  on r = a).
* ``cylinder_line_source``: line source H_0(k|rho - rho'|) parallel to the
  axis of an infinite circular cylinder:
      u^s = -sum [J_n(ka)/H_n(ka) | J_n'(ka)/H_n'(ka)] H_n(k rho') H_n(k rho) e^{jn(phi - phi')}
"""
import numpy as np
from scipy.special import hankel2, h2vp, jv, jvp, spherical_jn, spherical_yn


def _sph_h2(n, x, derivative=False):
    return spherical_jn(n, x, derivative) - 1j * spherical_yn(n, x, derivative)


def legendre_and_dtheta(nmax, theta):
    """P_n(cos th) and dP_n(cos th)/dth for n = 0..nmax (rows)."""
    x = np.cos(theta)
    s = np.sin(theta)
    P = np.zeros((nmax + 1,) + np.shape(theta))
    dP = np.zeros_like(P)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = x
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
    ssafe = np.where(np.abs(s) > 1e-300, s, 1.0)
    for n in range(1, nmax + 1):
        # (1 - x^2) P_n'(x) = n (P_{n-1} - x P_n);  d/dth = -sin(th) d/dx
        dP[n] = np.where(np.abs(s) > 1e-300, -n * (P[n - 1] - x * P[n]) / ssafe, 0.0)
    return P, dP


def _nmax(ka, kb, kr):
    return int(max(ka, 1.0) + 12 * max(ka, 1.0) ** (1 / 3) + 40)


def sphere_scalar(k, a, b, r, theta, hard=False, incident=True):
    """Total (or scattered, incident=False) field at (r, th); source on +z at b."""
    r = np.asarray(r, dtype=float)
    theta = np.asarray(theta, dtype=float)
    nmax = _nmax(k * a, k * b, k * np.max(r))
    n = np.arange(nmax + 1)
    P, _ = legendre_and_dtheta(nmax, theta)
    if hard:
        ratio = spherical_jn(n, k * a, True) / _sph_h2(n, k * a, True)
    else:
        ratio = spherical_jn(n, k * a) / _sph_h2(n, k * a)
    hb = _sph_h2(n, k * b)
    hr = np.stack([_sph_h2(nn, k * r) for nn in n])
    coef = 1j * k * (2 * n + 1) * ratio * hb
    us = np.einsum("n,n...->...", coef, hr * P)
    if not incident:
        return us
    R = np.sqrt(r * r + b * b - 2 * r * b * np.cos(theta))
    return us + np.exp(-1j * k * R) / R


def sphere_scalar_incident_series(k, b, r, theta, nmax):
    """The incident expansion alone (used to check the series conventions)."""
    n = np.arange(nmax + 1)
    P, _ = legendre_and_dtheta(nmax, theta)
    rl, rg = np.minimum(r, b), np.maximum(r, b)
    jl = np.stack([spherical_jn(nn, k * rl) for nn in n])
    hg = np.stack([_sph_h2(nn, k * rg) for nn in n])
    return np.einsum("n,n...->...", -1j * k * (2 * n + 1), jl * hg * P)


def _riccati_h_prime(n, x):
    return _sph_h2(n, x) + x * _sph_h2(n, x, True)


def _riccati_j_prime(n, x):
    return spherical_jn(n, x) + x * spherical_jn(n, x, True)


def radial_dipole_debye(k, b, r, theta, nmax, part):
    """(E_r, E_th) from the Debye series; part = 'incident' or 'scattered:a'."""
    n = np.arange(nmax + 1)
    P, dP = legendre_and_dtheta(nmax, theta)
    if part == "incident":
        rl, rg = np.minimum(r, b), np.maximum(r, b)
        # u_n = C_n z_n(k r) with z_n = j_n for r < b and h_n for r > b
        inner = r < b
        zn = np.stack([np.where(inner, spherical_jn(nn, k * r), _sph_h2(nn, k * r)) for nn in n])
        znp = np.stack([np.where(inner, spherical_jn(nn, k * r, True), _sph_h2(nn, k * r, True)) for nn in n])
        other = np.stack([np.where(inner, _sph_h2(nn, k * b), spherical_jn(nn, k * b)) for nn in n])
        C = (-1j * k * (2 * n + 1) / b)[:, None] * other
    else:
        a = float(part.split(":")[1])
        ratio = _riccati_j_prime(n, k * a) / _riccati_h_prime(n, k * a)
        zn = np.stack([_sph_h2(nn, k * r) for nn in n])
        znp = np.stack([_sph_h2(nn, k * r, True) for nn in n])
        C = (1j * k * (2 * n + 1) / b * ratio * _sph_h2(n, k * b))[:, None] * np.ones_like(zn)
    un = C * zn
    d_run = C * (zn + k * r * znp)          # d(r u_n)/dr
    nn1 = (n * (n + 1))[:, None]
    Er = np.sum(nn1 * un / r * P, axis=0)
    Eth = np.sum(d_run / r * dP, axis=0)
    return Er, Eth


def dipole_free_field(src, p, pts, k):
    """curl curl (p e^{-jkR}/R) at pts."""
    v = pts - src
    R = np.linalg.norm(v, axis=1)
    nh = v / R[:, None]
    pn = nh @ p
    far = k * k * (p[None, :] - pn[:, None] * nh) / R[:, None]
    near = (3 * pn[:, None] * nh - p[None, :]) * (1 / R ** 3 + 1j * k / R ** 2)[:, None]
    return (far + near) * np.exp(-1j * k * R)[:, None]


def sphere_radial_dipole(k, a, b, pts_sph, nmax=None):
    """Total E (spherical components E_r, E_th) for the radial dipole on +z at b,
    at points given as (r, th) pairs."""
    r, th = pts_sph[:, 0], pts_sph[:, 1]
    if nmax is None:
        nmax = _nmax(k * a, k * b, k * np.max(r))
    Er_s, Eth_s = radial_dipole_debye(k, b, r, th, nmax, "scattered:%r" % a)
    pts = np.stack([r * np.sin(th), np.zeros_like(r), r * np.cos(th)], 1)
    Ei = dipole_free_field(np.array([0.0, 0.0, b]), np.array([0.0, 0.0, 1.0]), pts, k)
    rhat = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1)
    thhat = np.stack([np.cos(th), np.zeros_like(th), -np.sin(th)], 1)
    Er_i = np.einsum("ij,ij->i", Ei, rhat)
    Eth_i = np.einsum("ij,ij->i", Ei, thhat)
    return Er_i + Er_s, Eth_i + Eth_s


def cylinder_line_source(k, a, rho_s, rho, phi, hard=False, incident=True):
    """Total field of the line source H_0(k|rho - rho_s|) at (rho_s, phi=0)."""
    rho = np.asarray(rho, dtype=float)
    phi = np.asarray(phi, dtype=float)
    nmax = int(k * a + 12 * max(k * a, 1) ** (1 / 3) + 40)
    n = np.arange(-nmax, nmax + 1)
    if hard:
        ratio = jvp(n, k * a) / h2vp(n, k * a)
    else:
        ratio = jv(n, k * a) / hankel2(n, k * a)
    hs = hankel2(n, k * rho_s)
    hr = np.stack([hankel2(nn, k * rho) for nn in n])
    ex = np.exp(1j * np.outer(n, np.atleast_1d(phi)).reshape((n.size,) + np.shape(phi)))
    us = -np.einsum("n,n...->...", ratio * hs, hr * ex)
    if not incident:
        return us
    d = np.sqrt(rho * rho + rho_s * rho_s - 2 * rho * rho_s * np.cos(phi))
    return us + hankel2(0, k * d)

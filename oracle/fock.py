"""Pekeris/Fock functions and the UTD transition function in FP64.

Test infrastructure (see ``oracle/__init__``).

The paper writes the shadow-region field as Eq. (4) and the reflected field as
Eq. (3) but only names the transfer and reflection dyadics (Sec. II-B).  Their
scalar kernels are the soft/hard Pekeris functions p*_s, p*_h of the
off-surface UTD (Pathak 1979; Pathak, Burnside and Marhefka 1980), time
convention e^{+j w t}:

    p*_s(xi) = e^{-j pi/4}/sqrt(pi) * Int V(t)/W2(t)  e^{-j xi t} dt
    p*_h(xi) = e^{-j pi/4}/sqrt(pi) * Int V'(t)/W2'(t) e^{-j xi t} dt

with the Fock-Airy functions V(t) = sqrt(pi) Ai(t),
W1,2(t) = 2 sqrt(pi) e^{+-j pi/6} Ai(t e^{+-j 2pi/3}).  The integral is Abel
regularised at t -> -inf, where the integrand tends to j/2; that produces the
singular part -e^{-j pi/4}/(2 sqrt(pi) xi), and

    Ptilde_p(xi) = p*_p(xi) + e^{-j pi/4}/(2 sqrt(pi) xi)

is an entire function of xi.

Three exact representations are evaluated numerically, each in the xi range
where it is well conditioned:

* xi >= XI_RESIDUE: the residue series over the zeros of W2 (creeping-wave
  modes), closing the contour in the lower half plane.
* XI_SADDLE <= xi < XI_RESIDUE: Ptilde by quadrature; the t < 0 half of the
  integral is rotated onto the ray t = -r e^{j psi} where W1/W2 decays.
* xi < XI_SADDLE (deep lit): with h = -(j/2) W1/W2 one has exactly
  p* = e^{-j pi/4}/sqrt(pi) * Int_{-inf}^{inf} h(t) e^{-j xi t} dt, and the
  real line is moved onto the straight steepest-descent line through the saddle
  t = -xi^2/4.  The result is returned as
  c_p(xi) = sqrt(-4/xi) e^{-j xi^3/12} p*_p(xi), which tends to +1 (soft) and
  -1 (hard).  For |xi| > XI_ASYMPTOTIC the two-term saddle-point expansion
  c_s = 1 + 2j/xi^3, c_h = -1 + 2j/xi^3 is used (derived below).

The transition function is that of Kouyoumjian and Pathak (1974):
F(X) = 2j sqrt(X) e^{jX} Int_{sqrt(X)}^inf e^{-j t^2} dt.
"""
import numpy as np
from scipy.special import airy, airye, ai_zeros, fresnel

SQPI = np.sqrt(np.pi)
E_MPI4 = np.exp(-1j * np.pi / 4)          # e^{-j pi/4}
ROT = np.exp(2j * np.pi / 3)              # e^{j 2pi/3}

XI_RESIDUE = 1.5      # residue series for xi >= this
XI_SADDLE = -5.0      # steepest-descent contour for xi < this
XI_ASYMPTOTIC = 300.0
X_ASYMPTOTIC = 50.0   # F(X) by its asymptotic series above this

# --------------------------------------------------------------------------
# Fock-Airy functions
# --------------------------------------------------------------------------


def fock_V(t):
    """V(t) = sqrt(pi) Ai(t) and V'(t)."""
    ai, aip, _, _ = airy(np.asarray(t, dtype=complex))
    return SQPI * ai, SQPI * aip


def fock_W1(t):
    """W1(t) = 2 sqrt(pi) e^{j pi/6} Ai(t e^{j 2pi/3}) and W1'(t)."""
    z = np.asarray(t, dtype=complex) * ROT
    ai, aip, _, _ = airy(z)
    c = 2 * SQPI * np.exp(1j * np.pi / 6)
    return c * ai, c * ROT * aip


def fock_W2(t):
    """W2(t) = 2 sqrt(pi) e^{-j pi/6} Ai(t e^{-j 2pi/3}) and W2'(t)."""
    z = np.asarray(t, dtype=complex) / ROT
    ai, aip, _, _ = airy(z)
    c = 2 * SQPI * np.exp(-1j * np.pi / 6)
    return c * ai, c * aip / ROT


# --------------------------------------------------------------------------
# Residue series (shadow side, xi > 0)
# --------------------------------------------------------------------------

N_RESIDUE = 80
_res_cache = {}


def residue_terms(hard):
    """Exponents z_n and weights w_n so that p*(xi) = sum_n w_n e^{z_n xi}.

    The poles of the integrand are the zeros of W2 (soft) or W2' (hard):
    t_n = alpha_n e^{-j pi/3} with Ai(-alpha_n) = 0, resp. Ai'(-beta_n) = 0.
    Closing clockwise in the lower half plane gives
    p*_s = -e^{-j pi/12}/(2 sqrt pi) sum e^{alpha_n e^{-j5pi/6} xi}/Ai'(-alpha_n)^2
    p*_h = -e^{-j pi/12}/(2 sqrt pi) sum e^{beta_n e^{-j5pi/6} xi}/(beta_n Ai(-beta_n)^2)
    (the residues follow from the Wronskian of Ai(z), Ai(z e^{-j2pi/3});
    the tests check the sum against the quadrature).
    """
    key = bool(hard)
    if key not in _res_cache:
        a, ap, ai, aip = ai_zeros(N_RESIDUE)
        rot = np.exp(-5j * np.pi / 6)
        if not hard:
            z = (-a) * rot
            w = 1.0 / aip ** 2
        else:
            z = (-ap) * rot
            w = 1.0 / ((-ap) * ai ** 2)
        w = -np.exp(-1j * np.pi / 12) / (2 * SQPI) * w
        _res_cache[key] = (z, w)
    return _res_cache[key]


def pstar_residue(xi, hard):
    """p*_p(xi) from the residue series; accurate for xi >= XI_RESIDUE."""
    xi = np.atleast_1d(np.asarray(xi, dtype=float))
    z, w = residue_terms(hard)
    return (w[None, :] * np.exp(np.outer(xi, z))).sum(axis=1)


# --------------------------------------------------------------------------
# Rotated-contour quadrature for Ptilde (moderate xi)
# --------------------------------------------------------------------------

PSI = np.pi / 12
_quad_cache = {}


def _panels(a, b, width, n):
    x, w = np.polynomial.legendre.leggauss(n)
    edges = np.linspace(a, b, int(round((b - a) / width)) + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    return ((hi - lo) / 2 * x + (hi + lo) / 2).ravel(), ((hi - lo) / 2 * w).ravel()


def _quad_nodes(hard):
    key = bool(hard)
    if key in _quad_cache:
        return _quad_cache[key]
    # t >= 0: integrand V/W2 (or V'/W2') decays like exp(-4/3 t^{3/2}).
    t, wt = _panels(0.0, 14.0, 0.25, 20)
    v, vp = fock_V(t)
    w2, w2p = fock_W2(t)
    g = vp / w2p if hard else v / w2
    # t < 0 rotated to t = -r e^{j psi}: h = -(j/2) W1/W2 decays like
    # exp(-4/3 r^{3/2} sin(3 psi/2)).
    r, wr = _panels(0.0, 40.0, 0.25, 20)
    tau = -r * np.exp(1j * PSI)
    w1, w1p = fock_W1(tau)
    w2, w2p = fock_W2(tau)
    h = -0.5j * (w1p / w2p if hard else w1 / w2)
    # first integral: kernel e^{-j xi t}; second: Int h(tau) e^{-j xi tau}
    # e^{j psi} dr with -j xi tau = j xi r e^{j psi}
    weights = np.concatenate([g * wt, h * np.exp(1j * PSI) * wr])
    exps = np.concatenate([-1j * t.astype(complex), 1j * r * np.exp(1j * PSI)])
    _quad_cache[key] = (exps, weights)
    return _quad_cache[key]


def ptilde_quad(xi, hard):
    """Ptilde_p(xi) by contour quadrature; accurate for -5 <= xi <= 2."""
    xi = np.atleast_1d(np.asarray(xi, dtype=float))
    exps, weights = _quad_nodes(hard)
    out = np.empty(xi.shape, dtype=complex)
    for s in range(0, xi.size, 512):
        blk = xi[s:s + 512]
        out[s:s + 512] = np.exp(np.outer(blk, exps)) @ weights
    return E_MPI4 / SQPI * out


def ptilde(xi, hard):
    """Ptilde_p(xi) = p*_p(xi) + e^{-j pi/4}/(2 sqrt(pi) xi) for xi >= XI_SADDLE."""
    xi = np.atleast_1d(np.asarray(xi, dtype=float))
    out = np.empty(xi.shape, dtype=complex)
    hi = xi >= XI_RESIDUE
    if hi.any():
        out[hi] = pstar_residue(xi[hi], hard) + E_MPI4 / (2 * SQPI * xi[hi])
    lo = ~hi
    if lo.any():
        out[lo] = ptilde_quad(xi[lo], hard)
    return out


def pstar(xi, hard):
    """p*_p(xi) for xi != 0 (not used near xi = 0, where it is singular)."""
    xi = np.atleast_1d(np.asarray(xi, dtype=float))
    out = np.empty(xi.shape, dtype=complex)
    hi = xi >= XI_RESIDUE
    if hi.any():
        out[hi] = pstar_residue(xi[hi], hard)
    deep = xi < XI_SADDLE
    if deep.any():
        x = xi[deep]
        out[deep] = c_lit(x, hard) * np.sqrt(-x / 4) * np.exp(1j * x ** 3 / 12)
    mid = ~(hi | deep)
    if mid.any():
        out[mid] = ptilde_quad(xi[mid], hard) - E_MPI4 / (2 * SQPI * xi[mid])
    return out


# --------------------------------------------------------------------------
# Deep lit: steepest-descent contour
# --------------------------------------------------------------------------

_GL_SD = np.polynomial.legendre.leggauss(160)


def c_lit(xi, hard):
    """c_p(xi) = sqrt(-4/xi) e^{-j xi^3/12} p*_p(xi) for xi < 0 (deep lit).

    Contour: t = -s0 + v e^{j pi/4}, s0 = xi^2/4, v real, which passes the
    saddle of h(t) e^{-j xi t} along its steepest-descent direction.  With
    s = -t = s0 (1 + x) and Lam = |xi|^3 the exponent of h e^{-j xi t} e^{-j xi^3/12}
    is j Lam (y-1)^2 (2y+1)/12, y = sqrt(1+x), evaluated in that factored form
    to avoid cancellation; the Airy ratio is taken from exponentially scaled
    Airy functions.  Near the saddle the integrand is Gaussian of width
    4/sqrt(Lam) in u = v/s0; the nodes cover +-6.5 widths (and at most
    |u| <= 3, where the exponent is below -0.4 Lam).

    For |xi| > XI_ASYMPTOTIC: saddle-point expansion to first order in 1/Lam.
    The phase function contributes the factor 1 - j/(3 Lam) (from its cubic
    and quartic Taylor terms, x^3/96 and x^4/256), the Airy ratio W1/W2
    contributes 1 - 2j u_1 * 12/Lam with u_1 = 5/72 (soft), resp. with
    v_1 = -7/72 for W1'/W2' (hard); together c_s = 1 + 2j/xi^3 and
    c_h = -1 + 2j/xi^3, the next terms being O(xi^-6).
    """
    xi = np.atleast_1d(np.asarray(xi, dtype=float))
    if np.any(xi >= 0):
        raise ValueError("c_lit needs xi < 0")
    out = np.empty(xi.shape, dtype=complex)
    big = np.abs(xi) > XI_ASYMPTOTIC
    if big.any():
        x = xi[big]
        out[big] = (-1.0 if hard else 1.0) + 2j / x ** 3
    sm = ~big
    if sm.any():
        x = xi[sm][:, None]
        lam = np.abs(x) ** 3
        s0 = x ** 2 / 4
        gx, gw = _GL_SD
        half = np.minimum(6.5 * 4 / np.sqrt(lam), 3.0)           # range in u
        u = half * gx[None, :]
        wu = half * gw[None, :]
        e4 = np.exp(1j * np.pi / 4)
        ratio = 1 - u * e4                                         # s/s0
        y = np.sqrt(ratio)
        ym1 = (ratio - 1) / (y + 1)
        expo = 1j * lam * ym1 ** 2 * (2 * y + 1) / 12
        tau = -s0 * ratio
        z1 = tau * ROT
        z2 = tau / ROT
        a1, a1p, _, _ = airye(z1)
        a2, a2p, _, _ = airye(z2)
        if hard:
            # W1'/W2' = e^{j pi/3} e^{j 4pi/3} Ai'(z1)/Ai'(z2); the scaled
            # derivatives carry the same exp(zeta) factors as Ai.
            rr = np.exp(1j * np.pi / 3) * np.exp(4j * np.pi / 3) * a1p / a2p
        else:
            rr = np.exp(1j * np.pi / 3) * a1 / a2
        # exp(-zeta1 + zeta2) (principal branches, as airye scales) equals
        # exp(j 4/3 s^{3/2}) on this contour segment (|u| <= 3 keeps
        # arg(z1) inside (-pi, pi)); it is folded into expo above.
        f = -0.5j * rr * np.exp(expo)
        integral = (f * wu).sum(axis=1) * s0[:, 0] * e4
        out[sm] = np.sqrt(-4 / xi[sm]) * E_MPI4 / SQPI * integral
    return out


# --------------------------------------------------------------------------
# Transition function
# --------------------------------------------------------------------------


def _fresnel_tail(u):
    """Int_u^inf e^{-j t^2} dt for u >= 0 via the Fresnel integrals C, S."""
    x = u * np.sqrt(2 / np.pi)
    S, C = fresnel(x)
    return np.sqrt(np.pi / 2) * ((0.5 - C) - 1j * (0.5 - S))


def _asym_terms(X, nterms=40):
    """Terms (-1)^n (2n-1)!!/(2jX)^n, n = 1..nterms, of the asymptotic series
    F(X) ~ sum_{n>=0} (-1)^n (2n-1)!!/(2jX)^n (repeated integration by parts of
    the Fresnel tail); used only for X > X_ASYMPTOTIC where the terms decrease
    far beyond nterms."""
    X = np.asarray(X, dtype=float)
    term = np.ones(X.shape, dtype=complex)
    acc = np.zeros(X.shape, dtype=complex)
    for n in range(1, nterms + 1):
        term = term * (-(2 * n - 1)) / (2j * X)
        acc = acc + term
    return acc


def transition_F(X):
    """F(X) for X >= 0."""
    X = np.atleast_1d(np.asarray(X, dtype=float))
    out = np.empty(X.shape, dtype=complex)
    big = X > X_ASYMPTOTIC
    if big.any():
        out[big] = 1.0 + _asym_terms(X[big])
    sm = ~big
    if sm.any():
        u = np.sqrt(X[sm])
        out[sm] = 2j * u * np.exp(1j * X[sm]) * _fresnel_tail(u)
    return out


def transition_F_over_sqrtX(X):
    """F(X)/sqrt(X), finite at X = 0 where it equals sqrt(pi) e^{j pi/4}."""
    X = np.atleast_1d(np.asarray(X, dtype=float))
    out = np.empty(X.shape, dtype=complex)
    big = X > X_ASYMPTOTIC
    if big.any():
        out[big] = (1.0 + _asym_terms(X[big])) / np.sqrt(X[big])
    sm = ~big
    if sm.any():
        u = np.sqrt(X[sm])
        out[sm] = 2j * np.exp(1j * X[sm]) * _fresnel_tail(u)
    return out


def one_minus_F(X):
    """1 - F(X), without cancellation for large X."""
    X = np.atleast_1d(np.asarray(X, dtype=float))
    out = np.empty(X.shape, dtype=complex)
    big = X > X_ASYMPTOTIC
    if big.any():
        out[big] = -_asym_terms(X[big])
    sm = ~big
    if sm.any():
        out[sm] = 1.0 - transition_F(X[sm])
    return out


# --------------------------------------------------------------------------
# UTD kernels used by the field assembly
# --------------------------------------------------------------------------


def shadow_B(xi, X, q, hard):
    """B_p(xi, X) = p*_p(xi) + e^{-j pi/4} (1 - F(X)) / (2 sqrt(pi) xi).

    This is the bracket of the creeping-wave coefficient
    T_p = -sqrt(m(Q1) m(Q2)) sqrt(2/k) B_p(xi^d, X^d) e^{-jkt} (PBM 1980),
    used for xi >= 0.  q = sqrt(X)/|xi| = sqrt(k L / 2)/m is passed separately
    so that the term F(X)/xi is evaluated as sgn(xi) q F(X)/sqrt(X), which stays
    finite at xi = 0 (sgn(0) = +1 on the shadow side).  Slightly negative xi
    (only reached when a gradient check freezes the classification) takes the
    same closed form.
    """
    xi = np.atleast_1d(np.asarray(xi, dtype=float))
    X = np.broadcast_to(np.asarray(X, dtype=float), xi.shape)
    q = np.broadcast_to(np.asarray(q, dtype=float), xi.shape)
    out = np.empty(xi.shape, dtype=complex)
    hi = xi >= XI_RESIDUE
    if hi.any():
        out[hi] = pstar_residue(xi[hi], hard) + E_MPI4 * one_minus_F(X[hi]) / (2 * SQPI * xi[hi])
    lo = ~hi
    if lo.any():
        sg = np.where(xi[lo] < 0, -1.0, 1.0)
        out[lo] = ptilde(xi[lo], hard) - E_MPI4 / (2 * SQPI) * sg * q[lo] * transition_F_over_sqrtX(X[lo])
    return out


def lit_Rbar(xi, X, q, hard):
    """Rbar_p = -e^{-j xi^3/12} B_p(xi, X), so that the UTD reflection
    coefficient is R_p = sqrt(-4/xi) Rbar_p (PBM 1980), used for xi <= 0.

    Rbar_p stays bounded as xi -> 0-, which lets the caller combine the
    singular sqrt(-4/xi) with the vanishing caustic distance rho_1.  F(X)/xi
    is evaluated as sgn(xi) q F(X)/sqrt(X) with sgn(0) = -1 on the lit side.
    Deep in the lit region p* is taken from c_lit:
    Rbar = -c sqrt(-xi)/2 - e^{-j xi^3/12} e^{-j pi/4} (1-F)/(2 sqrt(pi) xi).
    """
    xi = np.atleast_1d(np.asarray(xi, dtype=float))
    X = np.broadcast_to(np.asarray(X, dtype=float), xi.shape)
    q = np.broadcast_to(np.asarray(q, dtype=float), xi.shape)
    out = np.empty(xi.shape, dtype=complex)
    deep = xi < XI_SADDLE
    if deep.any():
        x = xi[deep]
        c = c_lit(x, hard)
        huge = np.abs(x) > 1e6
        xs = np.where(huge, -1.0, x)
        corr = np.exp(-1j * xs ** 3 / 12) * E_MPI4 * one_minus_F(X[deep]) / (2 * SQPI * xs)
        out[deep] = -c * np.sqrt(-x) / 2 - np.where(huge, 0.0, corr)
    mid = ~deep
    if mid.any():
        x = xi[mid]
        sg = np.where(x > 0, 1.0, -1.0)
        B = ptilde(x, hard) - E_MPI4 / (2 * SQPI) * sg * q[mid] * transition_F_over_sqrtX(X[mid])
        out[mid] = -np.exp(-1j * x ** 3 / 12) * B
    return out

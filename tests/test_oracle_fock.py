"""Pins of the oracle's Fock/Pekeris functions and transition function.

Each check ties the oracle to something other than itself: a printed table,
an independent exact representation of the same integral, a closed-form
limit, or a differential identity.
"""
import os

import numpy as np
import pytest

from oracle import fock

HERE = os.path.dirname(os.path.abspath(__file__))


def test_airy_zero_table():
    """Residue-series constants against A&S Table 10.13."""
    tab = np.loadtxt(os.path.join(HERE, "golden", "airy_zeros.txt"))
    from scipy.special import ai_zeros
    a, ap, ai, aip = ai_zeros(6)
    np.testing.assert_allclose(-a, tab[:, 1], atol=6e-9)
    np.testing.assert_allclose(aip, tab[:, 2], atol=6e-9)
    np.testing.assert_allclose(-ap, tab[:, 3], atol=6e-9)
    np.testing.assert_allclose(ai, tab[:, 4], atol=6e-9)
    # the weights used by the oracle are built from exactly these numbers
    z, w = fock.residue_terms(False)
    np.testing.assert_allclose(np.abs(z[:6]), tab[:, 1], rtol=1e-8)
    np.testing.assert_allclose(np.angle(z[:6]), -5 * np.pi / 6, atol=1e-15)
    np.testing.assert_allclose(np.abs(w[:6]), 1 / (2 * np.sqrt(np.pi) * tab[:, 2] ** 2), rtol=1e-7)
    z, w = fock.residue_terms(True)
    np.testing.assert_allclose(np.abs(z[:6]), tab[:, 3], rtol=1e-8)
    np.testing.assert_allclose(np.abs(w[:6]), 1 / (2 * np.sqrt(np.pi) * tab[:, 3] * tab[:, 4] ** 2), rtol=1e-7)


@pytest.mark.parametrize("hard", [False, True])
def test_residue_series_equals_contour_quadrature(hard):
    """Two exact representations of the same integral agree where both converge."""
    xi = np.linspace(0.6, 3.0, 25)
    quad = fock.ptilde_quad(xi, hard)
    res = fock.pstar_residue(xi, hard) + fock.E_MPI4 / (2 * fock.SQPI * xi)
    assert np.max(np.abs(quad - res)) < 2e-12


@pytest.mark.parametrize("hard", [False, True])
def test_steepest_descent_equals_rotated_ray(hard):
    """Deep-lit contour vs the rotated-ray quadrature on their overlap."""
    xi = np.linspace(-6.0, -5.0, 11)
    sd = fock.c_lit(xi, hard)
    ray = (fock.ptilde_quad(xi, hard) - fock.E_MPI4 / (2 * fock.SQPI * xi)) * np.sqrt(-4 / xi) * np.exp(-1j * xi ** 3 / 12)
    assert np.max(np.abs(sd - ray)) < 1e-12


@pytest.mark.parametrize("hard", [False, True])
def test_deep_lit_asymptotics(hard):
    """c_s -> 1 + 2j/xi^3, c_h -> -1 + 2j/xi^3 with an O(xi^-6) remainder:
    the saddle-point expansion checked against the contour integral, so
    R_s -> -1 and R_h -> +1 (the PEC geometrical-optics limit)."""
    xi = -np.array([20.0, 40.0, 80.0, 160.0, 290.0])
    c = fock.c_lit(xi, hard)
    lead = (-1.0 if hard else 1.0) + 2j / xi ** 3
    rem = np.abs(c - lead)
    assert np.all(rem < 40.0 / xi ** 6 + 2e-13)
    # the xi^-6 term is really there (and of the expected size) at moderate xi
    assert 5.0 < abs((c[0] - lead[0]) * xi[0] ** 6) < 40.0
    # beyond the switch the series is used; it joins the contour result
    xs = np.array([fock.XI_ASYMPTOTIC * -0.999, fock.XI_ASYMPTOTIC * -1.001])
    cs = fock.c_lit(xs, hard)
    lead = (-1.0 if hard else 1.0) + 2j / xs ** 3
    assert np.max(np.abs(cs - lead)) < 1e-13


def test_ptilde_at_zero():
    """Ptilde_p(0) has phase -pi/12 (soft) and pi - pi/12 (hard); values from
    the quadrature and from the residue series continued to xi = 0 agree."""
    ps = fock.ptilde(np.array([0.0]), False)[0]
    ph = fock.ptilde(np.array([0.0]), True)[0]
    assert abs(np.angle(ps) - (-np.pi / 12)) < 1e-12
    assert abs(np.angle(ph) - (np.pi - np.pi / 12)) < 1e-12
    np.testing.assert_allclose([ps, ph], [0.341999658 - 0.091638532j, -0.296703242 + 0.079501394j], atol=2e-9)


@pytest.mark.parametrize("hard", [False, True])
def test_lit_reflection_limits(hard):
    """R_p = sqrt(-4/xi) Rbar_p -> -1 (soft) / +1 (hard) deep in the lit
    region with F(X) -> 1."""
    xi = -np.array([8.0, 16.0, 50.0, 2000.0])
    X = np.full(xi.shape, 1e12)
    R = np.sqrt(-4 / xi) * fock.lit_Rbar(xi, X, np.ones_like(xi), hard)
    target = 1.0 if hard else -1.0
    err = np.abs(R - target)
    assert err[0] < 2e-2 and np.all(np.diff(err) < 0) and err[-1] < 1e-9


def test_transition_function_small_and_large_X():
    """F(X) against its small-X expansion (Kouyoumjian-Pathak) and its
    large-X asymptotic series, and F -> 1."""
    X = np.array([1e-6, 1e-4, 1e-3])
    small = (np.sqrt(np.pi * X) - 2 * X * np.exp(1j * np.pi / 4) - (2 / 3) * X ** 2 * np.exp(-1j * np.pi / 4)) \
        * np.exp(1j * (np.pi / 4 + X))
    assert np.max(np.abs(fock.transition_F(X) - small) / np.abs(small)) < 1e-5
    Xl = np.array([200.0, 1e3, 1e5])
    # F ~ 1 - 1/(2jX) + 3/(2jX)^2 - 15/(2jX)^3 (integration by parts)
    big = 1 - 1 / (2j * Xl) + 3 / (2j * Xl) ** 2 - 15 / (2j * Xl) ** 3
    assert np.max(np.abs(fock.transition_F(Xl) - big)) < 105 / (2 * Xl[0]) ** 4 * 1.01
    assert abs(fock.transition_F(np.array([1e8]))[0] - 1) < 1e-8


def test_transition_function_branches_join():
    """Fresnel-integral branch and asymptotic branch agree at the switch."""
    X = np.array([fock.X_ASYMPTOTIC * (1 - 1e-12), fock.X_ASYMPTOTIC * (1 + 1e-12)])
    u = np.sqrt(X)
    fres = 2j * u * np.exp(1j * X) * fock._fresnel_tail(u)
    asym = 1 + fock._asym_terms(X)
    assert np.max(np.abs(fres - asym)) < 1e-12


def test_transition_function_ode():
    """dF/dX = (j + 1/(2X)) F - j, from differentiating the definition."""
    X = np.array([0.05, 0.7, 3.0, 20.0, 80.0])
    h = 1e-5 * X
    dF = (fock.transition_F(X + h) - fock.transition_F(X - h)) / (2 * h)
    rhs = (1j + 1 / (2 * X)) * fock.transition_F(X) - 1j
    assert np.max(np.abs(dF - rhs)) < 1e-6


@pytest.mark.parametrize("hard", [False, True])
def test_shadow_B_branches_join(hard):
    """The two forms of B used on either side of XI_RESIDUE agree."""
    xi = np.array([fock.XI_RESIDUE - 1e-13, fock.XI_RESIDUE])
    for X in (0.3, 4.0, 300.0):
        q = np.sqrt(X) / xi
        B = fock.shadow_B(xi, np.full(2, X), q, hard)
        assert abs(B[0] - B[1]) < 1e-11


@pytest.mark.parametrize("hard", [False, True])
def test_lit_Rbar_branches_join(hard):
    xi = np.array([fock.XI_SADDLE - 1e-12, fock.XI_SADDLE])
    for X in (0.5, 30.0, 3e4):
        q = np.sqrt(X) / np.abs(xi)
        R = fock.lit_Rbar(xi, np.full(2, X), q, hard)
        assert abs(R[0] - R[1]) < 1e-11

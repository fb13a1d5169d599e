"""Pins for Bessel functions, Chebyshev coefficients and truncation orders.

Against: scipy.special.jv; the Jacobi-Anger expansion
exp(-i x cos th) = sum_n c_n(x) cos(n th); the Neumann sum rule; the
expansion-load values printed in Sec. II.A; brute force on the truncation
definition.
"""
import math

import numpy as np
import pytest
from scipy.special import jv

import oracle as o


@pytest.mark.parametrize("x", [1e-3, 0.5, 1.0, math.pi, 10.0, 32 * math.pi,
                               100.5, 256 * math.pi, 1024 * math.pi, 2048 * math.pi,
                               4096 * math.pi])
def test_bessel_matches_scipy(x):
    # single-block moment propagation over 2048 or 4096 steps needs
    # J_n(j pi) up to x = 4096 pi; both methods lose a few ulp per 1e3 orders
    nmax = o.truncation(x) + 10
    J = o.bessel_j(x, nmax)
    ref = jv(np.arange(nmax + 1), x)
    assert np.max(np.abs(J - ref)) < (1e-13 if x < 1000 else 2e-13)


def test_bessel_zero_argument():
    J = o.bessel_j(0.0, 5)
    assert J[0] == 1.0 and np.all(J[1:] == 0.0)


@pytest.mark.parametrize("x", [0.3, math.pi, 40 * math.pi])
def test_neumann_sum_rule(x):
    J = o.bessel_j(x, o.truncation(x) + 20)
    assert J[0] + 2 * np.sum(J[2::2]) == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("x", [math.pi, 8 * math.pi, 32 * math.pi])
def test_jacobi_anger_reconstructs_exponential(x):
    n = o.truncation(x)
    c = o.cheb_coeffs(x, n)
    theta = np.linspace(0.0, math.pi, 257)
    T = np.cos(np.outer(np.arange(n + 1), theta))      # T_n(cos th) = cos(n th)
    approx = c @ T
    exact = np.exp(-1j * x * np.cos(theta))
    assert np.max(np.abs(approx - exact)) < 1e-13


def test_coefficient_phases():
    c = o.cheb_coeffs(5.0, 8)
    J = jv(np.arange(9), 5.0)
    assert c[0] == pytest.approx(J[0], abs=1e-15)
    # c_n = 2 (-i)^n J_n: n=1 -> -2i J_1, n=2 -> -2 J_2, n=3 -> 2i J_3
    assert c[1] == pytest.approx(-2j * J[1], abs=1e-14)
    assert c[2] == pytest.approx(-2 * J[2], abs=1e-14)
    assert c[3] == pytest.approx(2j * J[3], abs=1e-14)
    assert c[4] == pytest.approx(2 * J[4], abs=1e-14)


@pytest.mark.parametrize("x", [math.pi, 4 * math.pi, 32 * math.pi, 100 * math.pi])
def test_truncation_definition_brute_force(x):
    eta = 1e-14
    N = o.truncation(x, eta)
    ref = jv(np.arange(N + 1), x)
    assert N > x
    assert 2 * abs(ref[N]) <= eta * 1.0001
    for n in range(int(math.floor(x)) + 1, N):
        assert 2 * abs(ref[n]) > eta * 0.9999


def test_truncation_values_of_dos_step():
    # N(pi) = 20 at eta = 1e-14; larger eta never needs more terms
    assert o.truncation(math.pi, 1e-14) == 20
    assert o.truncation(math.pi, 1e-7) < 20


def test_expansion_load_matches_paper(golden):
    g = golden("expansion_load.txt")
    eta, tol = float(g["eta"]), float(g["rel_tol"])
    R = lambda x: o.truncation(x, eta) / x
    Rpi = R(math.pi)
    assert Rpi == pytest.approx(float(g["R_pi"]), rel=tol)
    for k, key in ((4, "ratio_4pi"), (10, "ratio_10pi"), (25, "ratio_25pi"),
                   (100, "ratio_100pi")):
        assert R(k * math.pi) / Rpi == pytest.approx(float(g[key]), rel=tol)


def test_expansion_load_decreases():
    xs = [math.pi * b for b in (1, 2, 4, 8, 16, 32, 64, 128)]
    R = [o.truncation(x) / x for x in xs]
    assert all(a > b for a, b in zip(R, R[1:]))
    assert R[-1] > 1.0

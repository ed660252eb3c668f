"""Pins of the oracle's Boys function F_n(T) = int_0^1 t^{2n} exp(-T t^2) dt.

Checked against: the value at T = 0, the closed form of F_0 through erf, the
incomplete-gamma form evaluated by mpmath at 30 digits, direct mpmath
quadrature of the defining integral, the large-T asymptote, the downward
recursion and the derivative identity dF_n/dT = -F_{n+1}."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O

NMAX = 6
T_GRID = [0.0, 1e-12, 1e-6, 1e-3, 0.05, 0.3, 0.9, 1.7, 3.2, 5.0, 7.7, 11.0, 15.5,
          19.9, 24.0, 28.5, 29.999, 30.0, 30.001, 33.0, 40.0, 55.0, 80.0, 130.0, 200.0]


def mp_boys(n, T):
    mp.mp.dps = 30
    if T == 0:
        return mp.mpf(1) / (2 * n + 1)
    T = mp.mpf(T)
    return mp.gammainc(n + mp.mpf(1) / 2, 0, T) / (2 * T ** (n + mp.mpf(1) / 2))


def test_boys_at_zero():
    F = O.boys(NMAX, 0.0)
    for n in range(NMAX + 1):
        assert F[n] == 1.0 / (2 * n + 1)


@pytest.mark.parametrize("T", T_GRID)
def test_boys_incomplete_gamma(T):
    F = O.boys(NMAX, T)
    for n in range(NMAX + 1):
        ref = float(mp_boys(n, T))
        assert abs(F[n] - ref) <= 4e-15 * ref, (n, T, F[n], ref)


@pytest.mark.parametrize("T", [0.2, 4.0, 17.0, 29.0, 36.0, 90.0])
def test_boys_direct_quadrature(T):
    mp.mp.dps = 30
    F = O.boys(4, T)
    for n in range(5):
        ref = mp.quad(lambda t: t ** (2 * n) * mp.exp(-T * t * t), [0, 0.25, 0.5, 1])
        assert abs(F[n] - float(ref)) <= 4e-15 * float(ref)


def test_boys_f0_erf_closed_form():
    for T in np.geomspace(1e-4, 200.0, 200):
        ref = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
        assert abs(O.boys(0, T)[0] - ref) <= 3e-15 * ref


def test_boys_large_T_asymptote():
    for T in [60.0, 100.0, 500.0, 1e4, 1e8]:
        F = O.boys(NMAX, T)
        for n in range(NMAX + 1):
            dfac = np.prod(np.arange(2 * n - 1, 0, -2)) if n > 0 else 1.0
            ref = dfac / 2 ** (n + 1) * math.sqrt(math.pi / T ** (2 * n + 1))
            assert abs(F[n] - ref) <= 3e-15 * ref


def test_boys_downward_recursion():
    for T in np.geomspace(1e-3, 150.0, 60):
        F = O.boys(NMAX, T)
        for n in range(NMAX):
            rhs = (2 * T * F[n + 1] + math.exp(-T)) / (2 * n + 1)
            assert abs(F[n] - rhs) <= 1e-14 * F[n]


def test_boys_derivative():
    h = 1e-5
    for T in [0.01, 0.7, 6.0, 25.0, 31.0, 70.0]:
        d = (O.boys(NMAX, T + h) - O.boys(NMAX, T - h)) / (2 * h)
        F = O.boys(NMAX, T)
        assert np.allclose(d[:-1], -F[1:], rtol=1e-7, atol=0)

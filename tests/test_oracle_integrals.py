"""Pins of the oracle's Hermite E coefficients, R_{tuv} integrals, primitive
normalisation and overlaps, each against an independent route."""
import math

import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial.hermite import hermval

from oracle import oracle as O

from gauss_ref import Basis, gauss_moment, prim_norm as q_prim_norm


def _rand_pairs(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        a, b = np.exp(rng.uniform(np.log(0.1), np.log(20.0), 2))
        A, B = rng.uniform(-2, 2, 2)
        yield a, b, A, B


def test_E0_equals_binomial_overlap():
    """sqrt(pi/p) E^{ij}_0 is the 1-D overlap; the oracle computes the two by
    different expansions (E recursion vs binomial expansion about P)."""
    for a, b, A, B in _rand_pairs(40, 1):
        p = a + b
        for i in range(3):
            for j in range(3):
                e0 = O.hermite_E(i, j, 0, a, b, A, B)
                s = O.overlap1d(i, j, a, b, A, B)
                assert abs(math.sqrt(math.pi / p) * e0 - s) <= 1e-13 * (abs(s) + 1e-3)


def test_E_reproduces_gaussian_product():
    """(x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2) = sum_t E^{ij}_t Lambda_t(x)
    with Lambda_t = d^t/dP^t exp(-p (x-P)^2) = p^{t/2} H_t(sqrt(p)(x-P)) exp(...),
    H_t the physicists' Hermite polynomial (numpy hermval)."""
    for a, b, A, B in _rand_pairs(25, 2):
        p = a + b
        P = (a * A + b * B) / p
        xs = np.linspace(P - 2.5, P + 2.5, 21)
        for i in range(3):
            for j in range(3):
                lhs = (xs - A) ** i * (xs - B) ** j * np.exp(-a * (xs - A) ** 2 - b * (xs - B) ** 2)
                rhs = np.zeros_like(xs)
                for t in range(i + j + 1):
                    c = np.zeros(t + 1)
                    c[t] = 1.0
                    lam = p ** (t / 2) * hermval(math.sqrt(p) * (xs - P), c) * np.exp(-p * (xs - P) ** 2)
                    rhs += O.hermite_E(i, j, t, a, b, A, B) * lam
                scale = np.max(np.abs(lhs)) + 1e-300
                assert np.max(np.abs(lhs - rhs)) <= 1e-12 * scale + 1e-300


def _mp_F0(T):
    if T == 0:
        return mp.mpf(1)
    return mp.sqrt(mp.pi) / 2 * mp.erf(mp.sqrt(T)) / mp.sqrt(T)


@pytest.mark.parametrize("p,X,Y,Z", [(0.7, 0.4, -0.3, 0.9), (2.5, 1.1, 0.6, -0.5),
                                     (1.3, 3.0, -2.0, 4.5), (0.05, 0.2, 0.1, -0.1)])
def test_R_is_derivative_of_R000(p, X, Y, Z):
    """R^0_{tuv} = d^t/dX^t d^u/dY^u d^v/dZ^v F_0(p (X^2+Y^2+Z^2)), the
    derivatives taken by mpmath at 30 digits of the erf form of F_0."""
    mp.mp.dps = 30
    L = 4
    R = O.hermite_R(L, p, X, Y, Z)
    f = lambda x, y, z: _mp_F0(p * (x * x + y * y + z * z))
    for t in range(L + 1):
        for u in range(L + 1 - t):
            for v in range(L + 1 - t - u):
                ref = float(mp.diff(f, (X, Y, Z), (t, u, v)))
                scale = p ** ((t + u + v) / 2.0)
                assert abs(R[t, u, v] - ref) <= 1e-12 * scale, (t, u, v, R[t, u, v], ref)


def test_R_far_field_multipoles():
    """For p R^2 >= 60, (2 pi/p) R_{tuv} = (pi/p)^{3/2} d^t_X d^u_Y d^v_Z (1/R)
    up to an exponentially small tail."""
    mp.mp.dps = 30
    p = 1.7
    X, Y, Z = 4.0, -5.0, 3.5
    assert p * (X * X + Y * Y + Z * Z) >= 60
    R = O.hermite_R(4, p, X, Y, Z)
    f = lambda x, y, z: 1 / mp.sqrt(x * x + y * y + z * z)
    for t in range(5):
        for u in range(5 - t):
            for v in range(5 - t - u):
                ref = float((mp.pi / p) ** 1.5 * mp.diff(f, (X, Y, Z), (t, u, v)))
                got = 2 * math.pi / p * R[t, u, v]
                assert abs(got - ref) <= 1e-12 * abs(ref) + 1e-18


def test_primitive_normalisation():
    for a in [0.05, 0.3, 1.0, 7.0, 400.0]:
        for e in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (2, 0, 0), (1, 1, 0), (0, 1, 1)]:
            ref = q_prim_norm(a, e)
            assert abs(O.prim_norm(a, *e) - ref) <= 1e-13 * ref


def test_overlap_matrix_vs_quadrature():
    """Full contracted overlap matrix (s, p, d; two centres) against
    Gauss-Hermite quadrature of the test's own basis; diagonal = 1."""
    xyz = np.array([[0.1, 0.2, -0.3], [0.9, -0.6, 0.4]])
    shells = [(0, 0, [3.0, 0.8, 0.2], [0.3, 0.5, 0.4]), (0, 1, [1.1, 0.35], [0.6, 0.5]),
              (1, 2, [2.2, 0.4], [0.7, 0.4]), (1, 0, [0.5], [1.0])]
    flat = (np.array([s[0] for s in shells], np.int32), np.array([s[1] for s in shells], np.int32),
            np.array([len(s[2]) for s in shells], np.int32),
            np.cumsum([0] + [len(s[2]) for s in shells[:-1]]).astype(np.int64),
            np.concatenate([s[2] for s in shells]).astype(float),
            np.concatenate([s[3] for s in shells]).astype(float))
    S = O.overlap_matrix_raw(xyz, flat)
    Sq = Basis(xyz, shells).overlap()
    assert np.max(np.abs(S - Sq)) <= 1e-13
    assert np.allclose(np.diag(S), 1.0, rtol=0, atol=1e-14)

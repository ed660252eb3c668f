"""Pins of the oracle's field E = -grad V (CPU).

Independent routes: the closed form of a Gaussian charge plus a point
nucleus, fourth-order central differences of the (separately pinned) oracle
potential, Gauss's law div E = -4 pi rho_e with the density evaluated from
this file's own basis, the far-field monopole tr(P S), and invariances.  Two
planted mistakes (a transposed Hermite index, a flipped electronic sign)
must fail the difference pin."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1011_4687_amd import synth

from gauss_ref import Basis
from test_oracle_potential import SHELLS2, XYZ2, flat, rand_sym


def gaussian_charge_field(Z, q, p, A, pts):
    """E of a nucleus Z at A plus a normalised Gaussian electron cloud of q
    electrons and exponent p centred on A: V = Z/r - q erf(sqrt(p) r)/r, so
    E = [Z - q erf(sqrt(p) r) + 2 q sqrt(p/pi) r exp(-p r^2)] (r - A)/r^3."""
    d = pts - A
    out = np.zeros_like(d)
    for k, v in enumerate(d):
        r = math.sqrt(float(v @ v))
        x = math.sqrt(p) * r
        if x < 0.5:
            # erf(x) - 2 x exp(-x^2)/sqrt(pi) = (2/sqrt(pi)) sum_{n>=1} (-1)^(n+1) 2n x^(2n+1) / (n! (2n+1)),
            # summed directly: the difference of the two terms cancels to O(x^3)
            g = sum((-1) ** (n + 1) * 2 * n * x ** (2 * n + 1) / (math.factorial(n) * (2 * n + 1))
                    for n in range(1, 20))
            g *= 2.0 / math.sqrt(math.pi)
        else:
            g = math.erf(x) - 2.0 * x * math.exp(-x * x) / math.sqrt(math.pi)
        out[k] = (Z - q * g) * v / r ** 3
    return out


def test_s_gaussian_and_nucleus_closed_form():
    for a in [0.07, 0.9, 13.0, 900.0]:
        for Z, q in [(0.0, 1.0), (3.0, 0.37), (1.0, 1.0)]:
            A = np.array([0.2, -0.4, 0.5])
            pts = A + np.array([[0.01, 0, 0], [0.3, -0.2, 0.1], [2.0, 1.0, -1.0],
                                [10.0, 3.0, 4.0], [40.0, 0, 0], [0, -1e-3, 2e-3]])
            E, AE = O.field_raw(A[None], np.array([Z]), flat([(0, 0, [a], [1.0])]),
                                np.array([[q]]), pts)
            ref = gaussian_charge_field(Z, q, 2 * a, A, pts)
            err = np.abs(E - ref).max(axis=1)
            assert np.all(err <= 4e-15 * AE), (a, Z, q, err / AE)


def _fd_field(xyz, Z, shells, P, C, h):
    """-grad V by the fourth-order central difference of the oracle potential."""
    pts = []
    for d in range(3):
        for s in (-2, -1, 1, 2):
            e = np.zeros(3)
            e[d] = s * h
            pts.append(C + e)
    V, _, _, _ = O.potential_raw(xyz, Z, shells, P, np.array(pts))
    g = np.zeros(3)
    for d in range(3):
        fm2, fm1, fp1, fp2 = V[4 * d: 4 * d + 4]
        g[d] = (fm2 - 8 * fm1 + 8 * fp1 - fp2) / (12 * h)
    return -g


FD_POINTS = [(0.5, 0.4, 0.2), (0.36, -0.17, 0.12), (3.0, -2.0, 1.0), (1.2, 0.8, -1.6), (12.0, 3.0, -4.0),
             (0.7, 0.25, -0.45)]


@pytest.mark.parametrize("pt", FD_POINTS)
def test_field_is_minus_gradient_of_potential(pt):
    """s/p/d contracted two-centre system with nuclei and a general
    symmetric P: every component against differences of V (h = 1e-3)."""
    P = rand_sym(Basis(XYZ2, SHELLS2).nbf, 3)
    Z = np.array([6.0, 1.0])
    C = np.array(pt)
    E, AE = O.field_raw(XYZ2, Z, flat(SHELLS2), P, C[None])
    # step 1e-3 of the distance to the nearest nucleus (at most 1e-3 bohr):
    # the truncation error of the stencil grows like (h/d)^4 near 1/d
    h = 1e-3 * min(1.0, np.linalg.norm(XYZ2 - C, axis=1).min())
    ref = _fd_field(XYZ2, Z, flat(SHELLS2), P, C, h)
    assert np.abs(E[0] - ref).max() <= 1e-9 * AE[0], np.abs(E[0] - ref).max() / AE[0]


@pytest.mark.parametrize("mutation", [7, 8])
def test_planted_field_mistakes_are_caught(mutation):
    P = rand_sym(Basis(XYZ2, SHELLS2).nbf, 3)
    Z = np.array([6.0, 1.0])
    worst = 0.0
    for pt in FD_POINTS[:4]:
        C = np.array(pt)
        ref = _fd_field(XYZ2, Z, flat(SHELLS2), P, C, 1e-3)
        O.set_mutation(mutation)
        try:
            E, AE = O.field_raw(XYZ2, Z, flat(SHELLS2), P, C[None])
        finally:
            O.set_mutation(0)
        worst = max(worst, np.abs(E[0] - ref).max() / AE[0])
    assert worst > 1e-4


def test_gauss_law():
    """div E = -4 pi rho_e away from the nuclei (fourth-order differences of
    the oracle field; rho from this file's basis)."""
    B = Basis(XYZ2, SHELLS2)
    P = rand_sym(B.nbf, 5, psd=True)
    Z = np.array([6.0, 1.0])
    for C in [np.array([0.5, 0.1, -0.2]), np.array([0.9, 0.5, -0.4]), np.array([1.5, 1.0, -1.0])]:
        h = 1e-3
        pts = []
        for d in range(3):
            for s in (-2, -1, 1, 2):
                e = np.zeros(3)
                e[d] = s * h
                pts.append(C + e)
        E, _ = O.field_raw(XYZ2, Z, flat(SHELLS2), P, np.array(pts))
        div = 0.0
        for d in range(3):
            fm2, fm1, fp1, fp2 = E[4 * d: 4 * d + 4, d]
            div += (fm2 - 8 * fm1 + 8 * fp1 - fp2) / (12 * h)
        rho = B.density(P, C[None])[0]
        assert abs(div + 4 * math.pi * rho) <= 1e-8 * 4 * math.pi * rho, (div, -4 * math.pi * rho)


def test_far_field_monopole():
    """Far away E -> Q d / R^2 with Q = sum Z - tr(P S) (overlap by the
    binomial route); the half-difference of E at +-R d cancels the dipole."""
    env, _ = synth.workload("tiny", n_points=1)
    sc = O.neutral_scales(env) * 0.8
    q = O.fragment_electrons(env, scale=sc).sum()
    Q = env.Z.sum() - q
    d = np.array([0.36, -0.48, 0.8])
    R = 1e5
    E, AE = O.field(env, np.array([R * d, -R * d]), scale=sc)
    mono = 0.5 * (E[0] - E[1]) * R * R
    # the quadrupole part of the field is odd in d as well and survives the
    # half-difference: O((size/R)^2) relative, about 3e-8 here
    assert np.abs(mono - Q * d).max() <= 1e-7 * abs(Q)


def test_translation_and_linearity():
    B = Basis(XYZ2, SHELLS2)
    P, P2 = rand_sym(B.nbf, 7), rand_sym(B.nbf, 8)
    Z = np.array([6.0, 1.0])
    pts = np.array([[0.5, 0.2, -0.1], [2.0, -1.0, 3.0], [0.05, 0.0, 0.0]])
    E, AE = O.field_raw(XYZ2, Z, flat(SHELLS2), P, pts)
    shift = np.array([13.7, -4.2, 8.9])
    Es, _ = O.field_raw(XYZ2 + shift, Z, flat(SHELLS2), P, pts + shift)
    assert np.all(np.abs(Es - E).max(axis=1) <= 1e-12 * AE)
    E0, AE0 = O.field_raw(XYZ2, np.zeros(2), flat(SHELLS2), P, pts)
    E2, AE2 = O.field_raw(XYZ2, np.zeros(2), flat(SHELLS2), P2, pts)
    E3, _ = O.field_raw(XYZ2, np.zeros(2), flat(SHELLS2), 2.0 * P - 0.5 * P2, pts)
    assert np.all(np.abs(E3 - (2.0 * E0 - 0.5 * E2)).max(axis=1) <= 1e-13 * (AE0 + AE2))
    # nuclear part alone
    En, _ = O.field_raw(XYZ2, Z, flat(SHELLS2), None, pts)
    dv = pts[:, None, :] - XYZ2[None]
    r = np.linalg.norm(dv, axis=2)
    ref = (Z[None, :, None] * dv / r[:, :, None] ** 3).sum(axis=1)
    assert np.allclose(En, ref, rtol=1e-14, atol=0)

"""Pins of the oracle's whole potential V(r) = V_nuc - V_ele.

Independent routes: the erf closed form of an s Gaussian, the
Gaussian-transform quadrature of [mu nu|C] (tests/gauss_ref.py), brute-force
3-D quadrature of rho(r')/|r'-r|, Poisson's equation, far-field monopole =
tr(PS), and the invariances of the definition."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1011_4687_amd import synth

from gauss_ref import Basis, sphere_quadrature_potential


def flat(shells):
    return (np.array([s[0] for s in shells], np.int32),
            np.array([s[1] for s in shells], np.int32),
            np.array([len(s[2]) for s in shells], np.int32),
            np.cumsum([0] + [len(s[2]) for s in shells[:-1]]).astype(np.int64),
            np.concatenate([s[2] for s in shells]).astype(float),
            np.concatenate([s[3] for s in shells]).astype(float))


XYZ2 = np.array([[0.3, -0.2, 0.1], [1.1, 0.7, -0.9]])
SHELLS2 = [(0, 0, [2.1, 0.6], [0.5, 0.7]), (0, 1, [1.3, 0.4], [0.6, 0.3]),
           (1, 2, [1.7, 0.5], [0.4, 0.8]), (1, 1, [0.9], [1.0]), (0, 2, [1.1], [1.0]),
           (1, 0, [25.0, 4.0], [0.3, 0.6])]


def rand_sym(n, seed, psd=False):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((n, n))
    return (C @ C.T) * 0.05 if psd else (C + C.T) * 0.1


def test_s_gaussian_erf_closed_form():
    """A normalised s primitive squared is a Gaussian charge of exponent 2a:
    its potential is q erf(sqrt(2a) R)/R, and q 2 sqrt(2a/pi) at R = 0."""
    for a in [0.07, 0.9, 13.0, 900.0]:
        for q in [1.0, 0.37]:
            xyz = np.array([[0.2, -0.4, 0.5]])
            sh = [(0, 0, [a], [1.0])]
            pts = xyz + np.array([[0, 0, 0], [0.01, 0, 0], [0.3, -0.2, 0.1], [2.0, 1.0, -1.0],
                                  [10.0, 3.0, 4.0], [40.0, 0, 0]])
            _, _, Ve, _ = O.potential_raw(xyz, np.zeros(1), flat(sh), np.array([[q]]), pts)
            R = np.linalg.norm(pts - xyz, axis=1)
            ref = np.array([q * 2 * math.sqrt(2 * a / math.pi) if r == 0
                            else q * math.erf(math.sqrt(2 * a) * r) / r for r in R])
            assert np.allclose(Ve, ref, rtol=2e-15, atol=0)


def test_contracted_s_closed_form():
    """Contracted s: sum over primitive pairs of erf terms; the contraction scale
    is written here from the closed-form s overlap (pi/p)^{3/2}."""
    ex = np.array([5.0, 1.2, 0.3])
    co = np.array([0.2, 0.5, 0.6])
    n0 = (2 * ex / math.pi) ** 0.75
    S = sum(co[i] * co[j] * n0[i] * n0[j] * (math.pi / (ex[i] + ex[j])) ** 1.5
            for i in range(3) for j in range(3))
    xyz = np.zeros((1, 3))
    pts = np.array([[0.5, 0.1, 0.0], [2.0, 2.0, 1.0], [7.0, 0.0, 0.0]])
    _, _, Ve, _ = O.potential_raw(xyz, np.zeros(1), flat([(0, 0, ex, co)]), np.array([[1.0]]), pts)
    for k, pt in enumerate(pts):
        r = np.linalg.norm(pt)
        v = sum(co[i] * co[j] * n0[i] * n0[j] * (math.pi / (ex[i] + ex[j])) ** 1.5 *
                math.erf(math.sqrt(ex[i] + ex[j]) * r) / r for i in range(3) for j in range(3))
        assert abs(Ve[k] - v / S) <= 1e-14 * abs(v / S)


@pytest.mark.parametrize("pt", [(0.5, 0.4, 0.2), (0.3, -0.2, 0.1), (3.0, -2.0, 1.0),
                                (1.2, 0.8, -1.6), (12.0, 3.0, -4.0)])
def test_vele_vs_gaussian_transform_quadrature(pt):
    """s/p/d contracted two-centre system, general symmetric P: the oracle
    against quadrature of the Gaussian transform of 1/r (no Boys function, no
    Hermite recursion).  Points cover T from 0 to several hundred."""
    B = Basis(XYZ2, SHELLS2)
    P = rand_sym(B.nbf, 3)
    M = B.coulomb(np.array(pt))
    ref = float(np.sum(P * M))
    absref = float(np.sum(np.abs(P * M)))
    _, _, Ve, A = O.potential_raw(XYZ2, np.zeros(2), flat(SHELLS2), P, np.array([pt]))
    assert abs(Ve[0] - ref) <= 1e-12 * absref


def test_whole_potential_vs_3d_quadrature():
    """Brute force: V_ele(C) = int rho(r)/|r-C| d^3r in spherical coordinates
    around C with rho evaluated pointwise from the test's own basis."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.2, -0.5, 0.4]])
    shells = [(0, 0, [1.4, 0.5], [0.6, 0.5]), (0, 1, [0.8], [1.0]), (1, 2, [0.9, 0.45], [0.5, 0.6]),
              (1, 0, [0.7], [1.0])]
    B = Basis(xyz, shells)
    P = rand_sym(B.nbf, 11, psd=True)
    C = np.array([0.4, 0.3, -0.2])
    ref = sphere_quadrature_potential(B, P, C, s_max=13.0)
    _, _, Ve, _ = O.potential_raw(xyz, np.zeros(2), flat(shells), P, C[None])
    assert abs(Ve[0] - ref) <= 1e-9 * abs(ref)


def test_poisson_equation():
    """Laplacian of V_ele equals -4 pi rho (4th-order central differences)."""
    B = Basis(XYZ2, SHELLS2)
    P = rand_sym(B.nbf, 5, psd=True)
    for C in [np.array([0.5, 0.1, -0.2]), np.array([0.9, 0.5, -0.4])]:
        h = 0.01
        pts = [C]
        for d in range(3):
            for s in (-2, -1, 1, 2):
                e = np.zeros(3)
                e[d] = s * h
                pts.append(C + e)
        _, _, Ve, _ = O.potential_raw(XYZ2, np.zeros(2), flat(SHELLS2), P, np.array(pts))
        lap = 0.0
        for d in range(3):
            fm2, fm1, fp1, fp2 = Ve[1 + 4 * d: 5 + 4 * d]
            lap += (-fm2 + 16 * fm1 - 30 * Ve[0] + 16 * fp1 - fp2) / (12 * h * h)
        rho = B.density(P, C[None])[0]
        assert abs(lap + 4 * math.pi * rho) <= 2e-6 * 4 * math.pi * rho


def test_translation_and_linearity_and_permutation():
    B = Basis(XYZ2, SHELLS2)
    P = rand_sym(B.nbf, 7)
    P2 = rand_sym(B.nbf, 8)
    Z = np.array([6.0, 1.0])
    pts = np.array([[0.5, 0.2, -0.1], [2.0, -1.0, 3.0], [0.0, 0.0, 0.0]])
    V, Vn, Ve, A = O.potential_raw(XYZ2, Z, flat(SHELLS2), P, pts)
    shift = np.array([13.7, -4.2, 8.9])
    Vs, _, _, _ = O.potential_raw(XYZ2 + shift, Z, flat(SHELLS2), P, pts + shift)
    assert np.all(np.abs(Vs - V) <= 1e-13 * A)
    _, _, Ve2, A2 = O.potential_raw(XYZ2, Z, flat(SHELLS2), P2, pts)
    _, _, Ve3, _ = O.potential_raw(XYZ2, Z, flat(SHELLS2), 2.0 * P - 0.5 * P2, pts)
    assert np.all(np.abs(Ve3 - (2.0 * Ve - 0.5 * Ve2)) <= 1e-13 * (A + A2))
    # reverse the shell order (and permute P accordingly): same V
    order = list(range(len(SHELLS2)))[::-1]
    nb = [(s[1] + 1) * (s[1] + 2) // 2 for s in SHELLS2]
    start = np.cumsum([0] + nb)
    perm = np.concatenate([np.arange(start[k], start[k + 1]) for k in order])
    sh_r = [SHELLS2[k] for k in order]
    Vr, _, _, _ = O.potential_raw(XYZ2, Z, flat(sh_r), P[np.ix_(perm, perm)], pts)
    assert np.all(np.abs(Vr - V) <= 1e-13 * A)
    # nuclear part alone
    d = np.linalg.norm(pts[:, None, :] - XYZ2[None], axis=2)
    assert np.allclose(Vn, (Z / d).sum(axis=1), rtol=1e-15)


def test_far_field_monopole_is_trace_PS():
    """At large distance R V_ele -> tr(P S) (overlap by the binomial route,
    potential by the E/R route), and a neutral environment's V falls off
    faster than 1/R."""
    env, _ = synth.workload("tiny", n_points=1)
    sc = O.neutral_scales(env)
    q = O.fragment_electrons(env, scale=sc)
    assert abs(q.sum() - env.Z.sum()) <= 1e-12 * env.Z.sum()
    d = np.array([0.36, -0.48, 0.8])
    R = 1e6
    V, Vn, Ve, A = O.potential(env, np.array([R * d, -R * d]), scale=sc)
    # the average over +-R d cancels the dipole term; the quadrupole is O(1/R^2)
    assert abs(R * 0.5 * (Ve[0] + Ve[1]) - q.sum()) <= 1e-9 * q.sum()
    # neutral: R V -> 0 like 1/R (dipole) and R^2 V tends to a finite dipole term
    V2, _, _, _ = O.potential(env, np.array([1e3 * d, 1e4 * d]), scale=sc)
    assert abs(1e3 * V2[0]) <= 0.02 * q.sum()
    d1, d2 = 1e3 ** 2 * V2[0], 1e4 ** 2 * V2[1]
    assert abs(d1 - d2) <= 0.05 * abs(d2)


def test_point_on_nucleus_is_infinite():
    xyz = np.array([[0.0, 0.0, 0.0]])
    V, Vn, Ve, A = O.potential_raw(xyz, np.array([1.0]), flat([(0, 0, [1.0], [1.0])]),
                                   np.array([[1.0]]), xyz)
    assert np.isinf(V[0]) and V[0] > 0 and np.isfinite(Ve[0])


def test_screening_error_bound_mid():
    """The screening rule (threshold 1e-12) changes V by far less than 1e-6 Ha
    on the mid-size environment."""
    env, pts = synth.workload("mid", n_points=6)
    sc = O.neutral_scales(env)
    Vs, _, _, A = O.potential(env, pts, scale=sc, screen=True)
    Vf, _, _, _ = O.potential(env, pts, scale=sc, screen=False)
    assert np.max(np.abs(Vs - Vf)) <= 1e-6

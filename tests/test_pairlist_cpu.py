"""The host pair-list builder, isolated from the kernels: a test-side numpy
evaluation of the exported pairs (Boys function from scipy's incomplete gamma,
its own Hermite recursion) must reproduce the oracle to 1e-12 A(r).  A
builder bug (E coefficients, folding, screening, fragments) fails here on the
CPU; a kernel bug fails only the GPU parity tests."""
import math

import numpy as np
import pytest
from scipy.special import gamma, gammainc

from common import workload_scaled
from paper_1011_4687_amd import envpot as E


def boys_scipy(nmax, T):
    T = np.asarray(T, dtype=float)
    out = np.zeros((nmax + 1,) + T.shape)
    small = T < 1e-12
    Ts = np.where(small, 1.0, T)
    for n in range(nmax + 1):
        s = n + 0.5
        v = gammainc(s, Ts) * gamma(s) / (2.0 * Ts ** s)
        out[n] = np.where(small, 1.0 / (2 * n + 1) - T / (2 * n + 3), v)
    return out


def hermite_R_all(L, p, X, Y, Z):
    """R^0_{tuv} for all t+u+v <= L, arrays over pairs (test's own recursion)."""
    F = boys_scipy(L, p * (X * X + Y * Y + Z * Z))
    R = {}
    for n in range(L, -1, -1):
        R[(n, 0, 0, 0)] = (-2.0 * p) ** n * F[n]
        for t in range(L - n + 1):
            for u in range(L - n + 1 - t):
                for v in range(L - n + 1 - t - u):
                    if t + u + v == 0:
                        continue
                    if t:
                        r = X * R[(n + 1, t - 1, u, v)] + ((t - 1) * R[(n + 1, t - 2, u, v)] if t > 1 else 0)
                    elif u:
                        r = Y * R[(n + 1, t, u - 1, v)] + ((u - 1) * R[(n + 1, t, u - 2, v)] if u > 1 else 0)
                    else:
                        r = Z * R[(n + 1, t, u, v - 1)] + ((v - 1) * R[(n + 1, t, u, v - 2)] if v > 1 else 0)
                    R[(n, t, u, v)] = r
    return R


def comps(L):
    return [(t, u, v) for t in range(L + 1) for u in range(L + 1 - t) for v in range(L + 1 - t - u)]


def eval_pairs(Ls, cen, p, D, C):
    """sum over pairs of (2 pi/p) sum_tuv D_tuv R_tuv with D scaled by (pi/p)^{3/2}."""
    total = 0.0
    absum = 0.0
    for L in range(5):
        m = Ls == L
        if not m.any():
            continue
        X, Y, Z = (cen[m] - C).T
        R = hermite_R_all(L, p[m], X, Y, Z)
        acc = np.zeros(m.sum())
        for k, (t, u, v) in enumerate(comps(L)):
            acc += D[m, k] * R[(0, t, u, v)]
        acc *= 2.0 * np.sqrt(p[m] / math.pi)
        total += acc.sum()
        absum += np.abs(acc).sum()
    return total, absum


@pytest.mark.parametrize("name,npts,screening", [("tiny", 12, False), ("mid", 3, True)])
def test_exported_pairs_reproduce_oracle(name, npts, screening):
    from oracle import oracle as O
    env, pts, P, _ = workload_scaled(name)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    h = E.Environment(env.xyz, env.Z, env.fragment, shells, P, build_only=True,
                      screening=screening)
    Ls, g, cen, p, D = h.export_pairs()
    pts = pts[:npts]
    Vo, Vn, Ve, A = O.potential(env, pts, P=P, screen=screening)
    for i, C in enumerate(pts):
        ve, _ = eval_pairs(Ls, cen, p, D, C)
        assert abs(ve - Ve[i]) <= 1e-12 * A[i], (i, ve, Ve[i])

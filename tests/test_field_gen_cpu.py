"""The generated field code (csrc/field_gen.h), compiled for the host with
g++: the Hermite recursion to order L+1 and its contractions against the
oracle's own recursion, and the far-field polynomial derivatives against a
direct evaluation written here."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1011_4687_amd", "csrc")

HARNESS = r"""
#include <cmath>
#define __device__
#define __forceinline__ inline
using std::fma;
#include "field_gen.h"
extern "C" void near_field(int L, const double* G, double X, double Y, double Z, const double* D, double* o) {
  switch (L) {
    case 0: hermite_field_L0<double>(G, X, Y, Z, D, o); break;
    case 1: hermite_field_L1<double>(G, X, Y, Z, D, o); break;
    case 2: hermite_field_L2<double>(G, X, Y, Z, D, o); break;
    case 3: hermite_field_L3<double>(G, X, Y, Z, D, o); break;
    default: hermite_field_L4<double>(G, X, Y, Z, D, o); break;
  }
}
extern "C" void far_field(int L, const double* h, double x, double y, double z, double* o) {
  switch (L) {
    case 0: far_field_L0<double>(h, x, y, z, o); break;
    case 1: far_field_L1<double>(h, x, y, z, o); break;
    case 2: far_field_L2<double>(h, x, y, z, o); break;
    case 3: far_field_L3<double>(h, x, y, z, o); break;
    default: far_field_L4<double>(h, x, y, z, o); break;
  }
}
"""


@pytest.fixture(scope="module")
def gen(tmp_path_factory):
    d = tmp_path_factory.mktemp("fieldgen")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    so = d / "libh.so"
    subprocess.run(["g++", "-O1", "-ffp-contract=off", "-shared", "-fPIC", "-I", CSRC, str(src), "-o", str(so)],
                   check=True)
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.near_field.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.far_field.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    return lib


def comps(L):
    return [(t, u, v) for t in range(L + 1) for u in range(L + 1 - t) for v in range(L + 1 - t - u)]


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@pytest.mark.parametrize("L", range(5))
def test_near_recursion_against_oracle(gen, L):
    rng = np.random.default_rng(10 + L)
    for _ in range(20):
        p = float(rng.uniform(0.1, 20.0))
        X, Y, Z = rng.uniform(-1.5, 1.5, 3)
        F = O.boys(L + 1, p * (X * X + Y * Y + Z * Z))
        G = np.array([(-2.0 * p) ** n * F[n] for n in range(L + 2)])
        D = rng.standard_normal(len(comps(L)))
        o = np.zeros(4)
        gen.near_field(L, _p(G), X, Y, Z, _p(D), _p(o))
        R = O.hermite_R(L + 1, p, X, Y, Z)
        ref = np.zeros(4)
        scale = 0.0
        for k, (t, u, v) in enumerate(comps(L)):
            ref += D[k] * np.array([R[t, u, v], R[t + 1, u, v], R[t, u + 1, v], R[t, u, v + 1]])
            scale += abs(D[k]) * max(abs(R[t, u, v]), abs(R[t + 1, u, v]), abs(R[t, u + 1, v]),
                                     abs(R[t, u, v + 1]))
        assert np.abs(o - ref).max() <= 1e-13 * scale


@pytest.mark.parametrize("L", range(5))
def test_far_polynomial_and_derivatives(gen, L):
    rng = np.random.default_rng(20 + L)
    cs = comps(L)
    for _ in range(20):
        h = rng.standard_normal(len(cs))
        x, y, z = rng.uniform(-0.8, 0.8, 3)
        o = np.zeros(4)
        gen.far_field(L, _p(h), x, y, z, _p(o))
        H = sum(c * x ** a * y ** b * z ** g for c, (a, b, g) in zip(h, cs))
        dx = sum(c * a * x ** (a - 1) * y ** b * z ** g for c, (a, b, g) in zip(h, cs) if a > 0)
        dy = sum(c * b * x ** a * y ** (b - 1) * z ** g for c, (a, b, g) in zip(h, cs) if b > 0)
        dz = sum(c * g * x ** a * y ** b * z ** (g - 1) for c, (a, b, g) in zip(h, cs) if g > 0)
        scale = np.abs(h).sum() * 5
        assert np.abs(o - np.array([H, dx, dy, dz])).max() <= 1e-14 * scale

"""Independent numerical reference pieces for the oracle pins.

Nothing here shares code with ``oracle/`` or the library.  Everything is
evaluated by quadrature rather than by the closed forms the oracle uses:

* normalisation and overlaps by Gauss-Hermite quadrature (exact for a
  polynomial times a Gaussian);
* Coulomb integrals [mu nu | C] through the Gaussian transform
  1/|r - C| = (2/sqrt(pi)) int_0^inf exp(-t^2 |r - C|^2) dt, whose inner
  integrals factor into 1-D Gauss-Hermite sums and whose t integral is done
  by composite Gauss-Legendre quadrature (no Boys function, no Hermite
  recursion);
* the whole density rho(r) = sum P_{mu nu} chi_mu chi_nu evaluated pointwise,
  for 3-D quadrature and the Poisson check.

The only thing this module shares with the library is the *interface
convention*: Cartesian components in x-major order (p = x,y,z;
d = xx,xy,xz,yy,yz,zz), coefficients multiplying normalised primitives and
each contracted component renormalised to unit self-overlap.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.hermite import hermgauss
from numpy.polynomial.legendre import leggauss

GH_X, GH_W = hermgauss(24)


def comps(l):
    out = []
    for i in range(l, -1, -1):
        for j in range(l - i, -1, -1):
            out.append((i, j, l - i - j))
    return out


def gauss_moment(m, p):
    """integral x^m exp(-p x^2) dx by Gauss-Hermite quadrature."""
    y = GH_X / math.sqrt(p)
    return float(np.sum(GH_W * y ** m)) / math.sqrt(p)


def prim_norm(alpha, e):
    """1/sqrt(integral of (x^i y^j z^k e^{-alpha r^2})^2) by quadrature."""
    s = 1.0
    for d in range(3):
        s *= gauss_moment(2 * e[d], 2.0 * alpha)
    return 1.0 / math.sqrt(s)


def contracted_scale(exps, coefs, e):
    s = 0.0
    for a, ca in zip(exps, coefs):
        for b, cb in zip(exps, coefs):
            m = 1.0
            for d in range(3):
                m *= gauss_moment(2 * e[d], a + b)
            s += ca * cb * prim_norm(a, e) * prim_norm(b, e) * m
    return 1.0 / math.sqrt(s)


class Basis:
    """Flattened contracted Cartesian basis: one entry per component."""

    def __init__(self, xyz, shells):
        # shells: list of (atom, l, exps, coefs)
        self.funcs = []
        for (atom, l, exps, coefs) in shells:
            exps = np.asarray(exps, dtype=float)
            coefs = np.asarray(coefs, dtype=float)
            for e in comps(l):
                sc = contracted_scale(exps, coefs, e)
                w = np.array([sc * c * prim_norm(a, e) for a, c in zip(exps, coefs)])
                self.funcs.append((np.asarray(xyz[atom], dtype=float), e, exps, w))
        self.nbf = len(self.funcs)

    def values(self, pts):
        pts = np.asarray(pts, dtype=float).reshape(-1, 3)
        out = np.zeros((pts.shape[0], self.nbf))
        for k, (A, e, exps, w) in enumerate(self.funcs):
            d = pts - A
            r2 = np.sum(d * d, axis=1)
            poly = d[:, 0] ** e[0] * d[:, 1] ** e[1] * d[:, 2] ** e[2]
            rad = np.zeros(pts.shape[0])
            for a, c in zip(exps, w):
                rad += c * np.exp(-a * r2)
            out[:, k] = poly * rad
        return out

    def density(self, P, pts):
        v = self.values(pts)
        return np.einsum("ni,ij,nj->n", v, P, v)

    def overlap(self):
        S = np.zeros((self.nbf, self.nbf))
        for m, (A, ea, xa, wa) in enumerate(self.funcs):
            for n, (B, eb, xb, wb) in enumerate(self.funcs):
                s = 0.0
                for a, ca in zip(xa, wa):
                    for b, cb in zip(xb, wb):
                        f = 1.0
                        for d in range(3):
                            f *= _three_center_1d(ea[d], eb[d], a, b, 0.0, A[d], B[d], 0.0)
                        s += ca * cb * f
                S[m, n] = s
        return S

    def coulomb(self, C, t_nodes=None):
        """Matrix [mu nu | C] by the Gaussian-transform quadrature."""
        C = np.asarray(C, dtype=float)
        M = np.zeros((self.nbf, self.nbf))
        for m, (A, ea, xa, wa) in enumerate(self.funcs):
            for n in range(m, self.nbf):
                B, eb, xb, wb = self.funcs[n]
                s = 0.0
                for a, ca in zip(xa, wa):
                    for b, cb in zip(xb, wb):
                        s += ca * cb * _coulomb_prim(ea, eb, a, b, A, B, C)
                M[m, n] = M[n, m] = s
        return M


def _three_center_1d(i, j, a, b, g, A, B, C):
    """integral (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2 - g(x-C)^2) dx;
    g may be an array (one integral per entry)."""
    g = np.asarray(g, dtype=float)
    q = a + b + g
    Q = (a * A + b * B + g * C) / q
    K = np.exp(-(a * b * (A - B) ** 2 + a * g * (A - C) ** 2 + b * g * (B - C) ** 2) / q)
    x = Q[..., None] + GH_X / np.sqrt(q)[..., None]
    s = np.sum(GH_W * (x - A) ** i * (x - B) ** j, axis=-1)
    out = K / np.sqrt(q) * s
    return float(out) if out.ndim == 0 else out


def _t_rule(p, T):
    """Nodes/weights in t for int_0^inf f(t) dt, f ~ exp(-T u^2)-like in
    u = t/sqrt(p + t^2) (composite Gauss-Legendre, refined near u = 0)."""
    x, w = leggauss(24)
    # panel edges in u: geometric refinement around the width 1/sqrt(T)
    width = 1.0 / math.sqrt(max(T, 1.0))
    edges = [0.0]
    e = width / 8.0
    while e < 1.0:
        edges.append(e)
        e *= 1.6
    edges.append(1.0)
    us, ws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        us.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w)
    u = np.concatenate(us)
    wu = np.concatenate(ws)
    # t = sqrt(p) u / sqrt(1 - u^2), dt = sqrt(p) (1 - u^2)^{-3/2} du
    t = math.sqrt(p) * u / np.sqrt(1.0 - u * u)
    wt = wu * math.sqrt(p) * (1.0 - u * u) ** -1.5
    return t, wt


def _coulomb_prim(ea, eb, a, b, A, B, C):
    """integral g_a(r) g_b(r) / |r - C| d^3 r for unnormalised Cartesian
    primitives, by the Gaussian transform of 1/|r - C|."""
    p = a + b
    P = (a * A + b * B) / p
    T = p * float(np.sum((P - C) ** 2))
    t, wt = _t_rule(p, T)
    val = np.ones_like(t)
    for d in range(3):
        val = val * _three_center_1d(ea[d], eb[d], a, b, t * t, A[d], B[d], C[d])
    return 2.0 / math.sqrt(math.pi) * float(np.sum(wt * val))


def sphere_quadrature_potential(basis, P, C, s_max, n_r=160, n_theta=64, n_phi=128):
    """V_ele(C) = int rho(r)/|r - C| d^3r in spherical coordinates centred on C:
    int_0^s_max s ds int dOmega rho(C + s w) (Gauss-Legendre radial panels,
    Gauss-Legendre in cos(theta), trapezoid in phi)."""
    C = np.asarray(C, dtype=float)
    xr, wr = leggauss(n_r // 8)
    edges = np.linspace(0.0, s_max, 9)
    rs, rws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        rs.append(0.5 * (hi - lo) * xr + 0.5 * (hi + lo))
        rws.append(0.5 * (hi - lo) * wr)
    r = np.concatenate(rs)
    wr = np.concatenate(rws)
    ct, wct = leggauss(n_theta)
    ph = 2.0 * math.pi * np.arange(n_phi) / n_phi
    wph = np.full(n_phi, 2.0 * math.pi / n_phi)
    st = np.sqrt(1.0 - ct * ct)
    dirs = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(),
                     np.outer(ct, np.ones(n_phi)).ravel()], axis=1)
    wdir = np.outer(wct, wph).ravel()
    total = 0.0
    for k in range(r.shape[0]):
        pts = C + r[k] * dirs
        rho = basis.density(P, pts)
        total += wr[k] * r[k] * float(np.sum(wdir * rho))
    return total

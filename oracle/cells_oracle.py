"""FP64 CPU oracle of the paper's cell-sum form of the environment potential.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg
are the only callers.  Nothing in the product library imports this module.

The paper writes the electrostatic energy of an electron in the environment
as a sum over the nuclei and over the cells that carry the environment's
electron density (Sec. II.B, Eq. ElectrostaticField).  With the library's
sign convention (U_ES = -V):

    V(r) = sum_A Z_A / |r - R_A|  -  sum_m q_m / |r - r_m|,

q_m = rho(r_m) h^3 the electron count of cell m.  This is that definition
written out: every term in float64, each of the two sums accumulated in
extended precision (numpy long double), no reordering or blocking beyond
processing the points one at a time.
"""
from __future__ import annotations

import numpy as np


def potential(xyz, Z, cells, points):
    """(V, V_nuc, V_ele, A) at each point; A = V_nuc + sum_m |q_m| / |r - r_m|
    is the conditioning scale (the sum of the absolute values of all terms)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    Z = np.asarray(Z, dtype=np.float64).reshape(-1)
    cells = np.asarray(cells, dtype=np.float64).reshape(-1, 4)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    V = np.empty(n)
    Vn = np.empty(n)
    Ve = np.empty(n)
    A = np.empty(n)
    for i in range(n):
        p = pts[i]
        dn = np.sqrt(((xyz - p) ** 2).sum(axis=1))
        tn = Z / dn
        dc = np.sqrt(((cells[:, :3] - p) ** 2).sum(axis=1))
        tc = cells[:, 3] / dc
        vn = np.sum(tn.astype(np.longdouble))
        ve = np.sum(tc.astype(np.longdouble))
        Vn[i] = float(vn)
        Ve[i] = float(ve)
        V[i] = float(vn - ve)
        A[i] = float(np.sum(np.abs(tn).astype(np.longdouble)) + np.sum(np.abs(tc).astype(np.longdouble)))
    return V, Vn, Ve, A

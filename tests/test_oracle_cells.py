"""Pins of the cell-sum oracle (CPU) and of the cell workload generator.

The cell form has a plain definition (a sum of point-charge potentials), so
the oracle is pinned by what that definition fixes independently of the
code: single charges, exact symmetric arrangements, superposition, and the
continuum limit of a Gaussian density sampled on cells, whose potential
outside the density is q erf(sqrt(a) r)/r.
"""
import math

import numpy as np
import pytest

from oracle import cells_oracle as C
from paper_1011_4687_amd import synth


def test_single_cell_and_single_nucleus():
    p = np.array([[0.3, -1.2, 2.0]])
    V, Vn, Ve, A = C.potential([[1.0, 1.0, 1.0]], [7.0], [[-2.0, 0.5, 0.0, 1.5]], p)
    dn = math.dist(p[0], [1.0, 1.0, 1.0])
    dc = math.dist(p[0], [-2.0, 0.5, 0.0])
    assert Vn[0] == pytest.approx(7.0 / dn, rel=1e-15)
    assert Ve[0] == pytest.approx(1.5 / dc, rel=1e-15)
    assert V[0] == pytest.approx(7.0 / dn - 1.5 / dc, rel=1e-14)
    assert A[0] == pytest.approx(7.0 / dn + 1.5 / dc, rel=1e-15)


def test_cube_corners_exact():
    # eight equal charges on the corners of a cube of edge s centred on the point
    s, q = 0.8, 0.25
    c = np.array([[x, y, z, q] for x in (-s / 2, s / 2) for y in (-s / 2, s / 2) for z in (-s / 2, s / 2)])
    V, _, Ve, _ = C.potential(np.zeros((0, 3)), np.zeros(0), c, np.zeros((1, 3)))
    assert Ve[0] == pytest.approx(8 * q / (s * math.sqrt(3) / 2), rel=1e-15)
    assert V[0] == pytest.approx(-Ve[0], rel=1e-15)


def test_superposition_and_order():
    rng = np.random.default_rng(3)
    xyz = rng.uniform(-5, 5, (4, 3))
    Z = np.array([1.0, 6.0, 7.0, 8.0])
    cells = np.concatenate([rng.uniform(-5, 5, (300, 3)), rng.uniform(0, 0.1, (300, 1))], axis=1)
    pts = rng.uniform(-1, 1, (5, 3)) + 10.0
    V, _, _, _ = C.potential(xyz, Z, cells, pts)
    V1, _, _, _ = C.potential(xyz, Z, cells[:150], pts)
    V2, _, _, _ = C.potential(np.zeros((0, 3)), np.zeros(0), cells[150:], pts)
    np.testing.assert_allclose(V, V1 + V2, rtol=0, atol=1e-13)
    perm = rng.permutation(len(cells))
    Vp, _, _, _ = C.potential(xyz[::-1], Z[::-1], cells[perm], pts)
    np.testing.assert_allclose(V, Vp, rtol=0, atol=1e-13)
    # translation of everything
    t = np.array([3.0, -7.0, 1.5])
    Vt, _, _, _ = C.potential(xyz + t, Z, np.concatenate([cells[:, :3] + t, cells[:, 3:]], axis=1), pts + t)
    np.testing.assert_allclose(V, Vt, rtol=0, atol=1e-12)


def _gaussian_cells(alpha, q, h, extent):
    ax = np.arange(-extent, extent + 0.5 * h, h)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    rho = q * (alpha / math.pi) ** 1.5 * np.exp(-alpha * (g ** 2).sum(axis=1))
    return np.concatenate([g, (rho * h ** 3)[:, None]], axis=1)


def test_continuum_limit_is_the_erf_potential():
    """Cells sampling a normalised Gaussian density converge to its exact
    potential q erf(sqrt(a) r)/r: fast outside the density, at second order
    in h inside it (the singular cell aside; the point lies between grid
    planes)."""
    alpha, q = 1.3, 2.0
    outside = np.array([[2.5, 0.0, 2.5], [0.0, -3.3, 1.1]])
    inside = np.array([[0.0713, 0.0491, 1.0137]])
    errs_out, errs_in = [], []
    for h in (0.3, 0.15):
        cells = _gaussian_cells(alpha, q, h, 5.2)
        for pts, errs in ((outside, errs_out), (inside, errs_in)):
            r = np.linalg.norm(pts, axis=1)
            exact = np.array([q * math.erf(math.sqrt(alpha) * x) / x for x in r])
            _, _, Ve, _ = C.potential(np.zeros((0, 3)), np.zeros(0), cells, pts)
            errs.append(np.abs(Ve - exact).max())
    assert errs_out[0] < 1e-7 and errs_out[1] < 1e-8
    assert errs_in[1] < 0.4 * errs_in[0]


def test_cell_workload_shape():
    env, pts = synth.cell_workload(n_points=512)
    assert len(env.Z) == 19
    assert 250_000 < env.n_cells < 290_000
    assert env.cells[:, 3].sum() == pytest.approx(env.Z.sum(), rel=1e-12)
    assert np.all(env.cells[:, 3] > 0)
    assert np.all(np.linalg.norm(pts, axis=1) <= 3.0)
    d = np.sqrt(((pts[:64, None, :] - env.cells[None, :, :3]) ** 2).sum(axis=2)).min()
    assert d >= 0.5
    env2, pts2 = synth.cell_workload(n_points=512)
    assert synth.digest(env.cells, pts) == synth.digest(env2.cells, pts2)

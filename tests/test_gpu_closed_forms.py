"""GPU results against closed forms, with no oracle in between.

* One atom carrying one normalised s Gaussian with density matrix q: the
  density is q (2a/pi)^{3/2} exp(-2a r^2), so
  V(r) = Z/r - q erf(sqrt(2a) r)/r   (and Z - q at large r, 2 q sqrt(2a/pi)
  subtracted at r -> 0).
* A zero density matrix leaves the point charges: V = sum_A Z_A / |r - R_A|.
Points cover p r^2 from 1e-6 to 4e3, across the near/far switch of both
precisions."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _gpu(E, pts):
    import torch
    v = E.eval(torch.from_numpy(np.ascontiguousarray(pts)).cuda())
    torch.cuda.synchronize()
    return v.cpu().numpy()


def _radial_points(center, rmin, rmax, n, seed):
    rng = np.random.default_rng(seed)
    r = np.exp(rng.uniform(np.log(rmin), np.log(rmax), n))
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    return center + r[:, None] * u, r


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("alpha", [0.08, 1.7, 950.0])
def test_single_s_gaussian_erf(precision, alpha):
    from paper_1011_4687_amd.envpot import Environment
    print(f"[closed] s gaussian {precision} alpha={alpha}", flush=True)
    A = np.array([[1.25, -0.5, 2.0]])
    Z, q = 6.0, 1.7
    p = 2.0 * alpha
    pts, _ = _radial_points(A[0], 1e-3 / math.sqrt(p), 60.0 / math.sqrt(p) + 1.0, 4097, 7)
    r = np.linalg.norm(pts - A[0], axis=1)   # the distance the stored points really have
    E = Environment(A, [Z], [0], [(0, 0, np.array([alpha]), np.array([1.0]))], np.array([[q]]),
                    precision=precision, screening=False)
    V = _gpu(E, pts)
    ref = np.array([Z / x - q * math.erf(math.sqrt(p) * x) / x for x in r])
    scale = Z / r + q / r   # sum of |terms|
    err = np.abs(V - ref)
    if precision == "fp64":
        assert np.all(err <= 2e-15 * scale), (err / scale).max()
    else:
        # relative to sum|terms|: points a few 1e-5 bohr from the nucleus carry
        # potentials of 1e5 hartree, where only the relative error is meaningful
        assert np.all(err <= 2e-7 * scale), (err / scale).max()
    E.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_zero_density_is_point_charges(precision):
    from paper_1011_4687_amd import synth
    from paper_1011_4687_amd.envpot import Environment
    print(f"[closed] zero density {precision}", flush=True)
    env, pts = synth.workload("tiny", n_points=1000)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    nbf = env.nbf
    E = Environment(env.xyz, env.Z, env.fragment, shells, np.zeros((nbf, nbf)), precision=precision)
    assert E.info()["n_pairs"] == 0
    V = _gpu(E, pts)
    d = np.linalg.norm(pts[:, None, :] - env.xyz[None, :, :], axis=2)
    ref = (env.Z[None, :] / d).sum(axis=1)
    assert np.all(np.abs(V - ref) <= 1e-14 * ref)
    E.close()

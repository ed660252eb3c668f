"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

FP64 path: |V_gpu - V_oracle(screened)| <= 1e-12 A(r), A(r) = V_nuc + sum|terms|
FP32C path: |V_gpu - V_oracle(full)| <= 1e-5 hartree (absolute)."""
import numpy as np
import pytest

from common import sample_indices, workload_scaled

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP64_REL = 1e-12


def _env(name, precision, n_points=None, screening=True):
    from paper_1011_4687_amd.envpot import Environment
    env, pts, P, _ = workload_scaled(name, n_points)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    return Environment(env.xyz, env.Z, env.fragment, shells, P, precision=precision,
                       screening=screening), env, pts, P


def _gpu(E, pts):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    v = E.eval(x)
    torch.cuda.synchronize()
    return v.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_tiny_all_points(precision):
    from oracle import oracle as O
    print(f"[parity] tiny {precision}", flush=True)
    E, env, pts, P = _env("tiny", precision, screening=False)
    V = _gpu(E, pts)
    Vo, Vn, Ve, A = O.potential(env, pts, P=P, screen=False)
    err = np.abs(V - Vo)
    if precision == "fp64":
        assert np.all(err <= FP64_REL * A), (err / A).max()
    else:
        assert err.max() <= FP32_TOL, err.max()
    E.close()


def _golden(name, env, pts):
    """Stored oracle values (tests/golden/<name>, written by
    tests/golden/make_goldens.py from the oracle alone) for this workload."""
    import os
    from paper_1011_4687_amd import synth
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not written yet")
    g = dict(np.load(path))
    assert str(g["env_digest"]) == env.digest() and str(g["points_digest"]) == synth.digest(pts)
    return g


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_mid_full_size_sampled(precision):
    """The mid workload at its full size (131072 points, the benchmark's
    launch configuration) against the stored screened-oracle values at
    16,384 seeded-random points; FP32C also against the unscreened oracle on
    32 of them (the screening error is inside the 1e-5 Ha budget)."""
    from oracle import oracle as O
    print(f"[parity] mid {precision}", flush=True)
    E, env, pts, P = _env("mid", precision)
    V = _gpu(E, pts)
    g = _golden("mid_oracle_16384.npz", env, pts)
    idx, Vo, A = g["idx"], g["V"], g["A"]
    err = np.abs(V[idx] - Vo)
    print(f"[parity] mid {precision}: max {err.max():.3e} Ha, rms {np.sqrt(np.mean(err ** 2)):.3e}, "
          f"max/A {(err / A).max():.3e} on {len(idx)} points", flush=True)
    if precision == "fp64":
        assert np.all(err <= FP64_REL * A), (err / A).max()
    else:
        assert err.max() <= FP32_TOL
        sub = idx[:: len(idx) // 32][:32]
        Vf, _, _, _ = O.potential(env, pts[sub], P=P, screen=False)
        assert np.abs(V[sub] - Vf).max() <= FP32_TOL
    E.close()


def test_mid_fp32c_against_fp64_every_point():
    """Every point of the full mid launch: FP32C against the FP64 kernel
    (which the oracle pins at 1e-12 A), so the FP32C error tail is seen on all
    131,072 points, not only on the oracle's sample."""
    print("[parity] mid fp32c vs fp64, all points", flush=True)
    E32, env, pts, P = _env("mid", "fp32c")
    E64, _, _, _ = _env("mid", "fp64")
    d = np.abs(_gpu(E32, pts) - _gpu(E64, pts))
    print(f"[parity] mid fp32c - fp64: max {d.max():.3e}, rms {np.sqrt(np.mean(d ** 2)):.3e}", flush=True)
    assert d.max() <= FP32_TOL
    E32.close()
    E64.close()


@pytest.mark.parametrize("n", [1, 63, 255, 257, 1000, 4097])
def test_ragged_sizes(n):
    """Point counts that leave ragged tails in the last wave/block and that
    select different split factors."""
    from oracle import oracle as O
    print(f"[parity] ragged n={n}", flush=True)
    E64, env, pts, P = _env("tiny", "fp64", n_points=n, screening=False)
    E32, _, _, _ = _env("tiny", "fp32c", n_points=n, screening=False)
    V64 = _gpu(E64, pts)
    V32 = _gpu(E32, pts)
    Vo, _, _, A = O.potential(env, pts, P=P, screen=False)
    assert np.all(np.abs(V64 - Vo) <= FP64_REL * A)
    assert np.abs(V32 - Vo).max() <= FP32_TOL
    E64.close()
    E32.close()


def test_zero_points_and_determinism():
    import torch
    E, env, pts, P = _env("tiny", "fp32c", screening=False)
    x = torch.from_numpy(pts).cuda()
    out = torch.full((0,), 1.0, dtype=torch.float64, device="cuda")
    E.eval(x[:0], out=out)
    a = E.eval(x).cpu().numpy()
    b = E.eval(x).cpu().numpy()
    assert np.array_equal(a, b)
    E.close()


def test_point_on_nucleus_is_inf():
    E, env, pts, P = _env("tiny", "fp64", screening=False)
    V = _gpu(E, env.xyz[:3])
    assert np.all(np.isposinf(V))
    E.close()


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_clusters_match_pairwise(precision):
    """Same-centre clusters change only the rounding: on every point of the
    full mid workload the merged evaluation agrees with the pair-by-pair one
    (waves with some point inside a cluster's radius take its members), and
    the sampled points agree with the oracle."""
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Environment
    print(f"[parity] clusters {precision}", flush=True)
    env, pts, P, _ = workload_scaled("mid", None)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    Em = Environment(env.xyz, env.Z, env.fragment, shells, P, precision=precision)
    Ep = Environment(env.xyz, env.Z, env.fragment, shells, P, precision=precision, merge=False)
    assert Em.info()["n_clusters"] > 0 and Ep.info()["n_clusters"] == 0
    Vm, Vp = _gpu(Em, pts), _gpu(Ep, pts)
    d = np.abs(Vm - Vp)
    print(f"[parity] clusters {precision}: max |merged - pairwise| {d.max():.3e}", flush=True)
    assert d.max() <= (2e-6 if precision == "fp32c" else 1e-11)
    idx = sample_indices(len(pts), 24)
    Vo, _, _, A = O.potential(env, pts[idx], P=P, screen=precision == "fp64")
    if precision == "fp64":
        assert np.all(np.abs(Vm[idx] - Vo) <= FP64_REL * A)
    else:
        assert np.abs(Vm[idx] - Vo).max() <= FP32_TOL
    Em.close()
    Ep.close()


@pytest.mark.parametrize("precision,shapes", [
    ("fp32c", [(4, 0), (4, 3), (4, 6), (4, 8), (2, 5), (1, 2)]),
    ("fp64", [(2, 0), (2, 6), (2, 8), (1, 3)]),
])
def test_launch_shapes_agree(precision, shapes, monkeypatch):
    """Every points-per-lane / pair-split shape gives the same potential up to
    rounding: splits cut ordinary and cluster segments at different places,
    and each shape is bitwise reproducible."""
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Environment
    print(f"[parity] shapes {precision}", flush=True)
    env, pts, P, _ = workload_scaled("mid", 8192)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    E = Environment(env.xyz, env.Z, env.fragment, shells, P, precision=precision)
    ref = _gpu(E, pts)
    idx = sample_indices(len(pts), 6)
    Vo, _, _, A = O.potential(env, pts[idx], P=P, screen=precision == "fp64")
    for np_, k in shapes:
        monkeypatch.setenv("ENVPOT_NP", str(np_))
        monkeypatch.setenv("ENVPOT_SPLIT_LOG2", str(k))
        V1 = _gpu(E, pts)
        V2 = _gpu(E, pts)
        assert np.array_equal(V1, V2), (np_, k)
        d = np.abs(V1 - ref).max()
        if precision == "fp64":
            assert d <= 1e-11, (np_, k, d)
            assert np.all(np.abs(V1[idx] - Vo) <= FP64_REL * A), (np_, k)
        else:
            assert d <= 2e-6, (np_, k, d)
            assert np.abs(V1[idx] - Vo).max() <= FP32_TOL, (np_, k)
    E.close()


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_morton_order_matches_caller_order(precision, monkeypatch):
    """Calls of 32,768 points or more are evaluated in Morton order and
    scattered back: around the threshold (32767, 32768, 40001 points) the
    values match the caller-order evaluation to rounding, the potential and
    the field agree, and both are bitwise repeatable."""
    import torch
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Environment
    print(f"[parity] morton order {precision}", flush=True)
    env, pts, P, _ = workload_scaled("mid", 40001)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    E = Environment(env.xyz, env.Z, env.fragment, shells, P, precision=precision)
    tol = 2e-6 if precision == "fp32c" else 1e-11
    for n in (32767, 32768, 40001):
        x = torch.from_numpy(np.ascontiguousarray(pts[:n])).cuda()
        monkeypatch.delenv("ENVPOT_NO_SORT", raising=False)
        V1 = _gpu(E, pts[:n])
        assert np.array_equal(V1, _gpu(E, pts[:n]))
        F1 = E.eval_field(x).cpu().numpy()
        monkeypatch.setenv("ENVPOT_NO_SORT", "1")
        V0 = _gpu(E, pts[:n])
        F0 = E.eval_field(x).cpu().numpy()
        assert np.abs(V1 - V0).max() <= tol, (n, np.abs(V1 - V0).max())
        assert np.abs(F1 - F0).max() <= tol, (n, np.abs(F1 - F0).max())
        assert np.abs(F1[:, 0] - V1).max() <= 2 * tol + (2e-6 if precision == "fp32c" else 0.0)
    idx = sample_indices(40001, 6)
    Vo, _, _, A = O.potential(env, pts[idx], P=P, screen=precision == "fp64")
    if precision == "fp64":
        assert np.all(np.abs(V1[idx] - Vo) <= FP64_REL * A)
    else:
        assert np.abs(V1[idx] - Vo).max() <= FP32_TOL
    E.close()

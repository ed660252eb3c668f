"""The library's host evaluation (ENV_FORCE_CPU: the paper's switch back to
the CPU, Sec. I) against the FP64 oracle, in this container with no GPU.

The host path evaluates the library's own screened pair list (its own Boys
tables, far-field coefficients and generated Hermite recursion), so these
tests pin the pair-list builder and the FP64 arithmetic of the method with no
kernel in between: |V_host - V_oracle| <= 1e-12 A(r) per point, A the
oracle's conditioning scale (nuclear term plus the sum of |terms|)."""
import os

import numpy as np
import pytest

from common import sample_indices, workload_scaled
from paper_1011_4687_amd import envpot as E


def _host(env, P, **kw):
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    return E.Environment(env.xyz, env.Z, env.fragment, shells, P, precision="fp64", force_cpu=True, **kw)


@pytest.mark.parametrize("screening", [False, True])
def test_tiny_all_points(screening):
    from oracle import oracle as O
    env, pts, P, _ = workload_scaled("tiny")
    h = _host(env, P, screening=screening)
    info = h.info()
    assert info["on_host"] == 1 and info["built_on_device"] == 0 and info["device_bytes"] == 0
    V = h.eval_host(pts)
    Vo, _, _, A = O.potential(env, pts, P=P, screen=screening)
    err = np.abs(V - Vo)
    print(f"tiny host (screening={screening}): max |dV|/A {(err / A).max():.2e}, max |dV| {err.max():.2e}")
    assert np.all(err <= 1e-12 * A)


@pytest.mark.parametrize("merge", [True, False])
def test_mid_sampled(merge):
    """Contracted s/p/d shells, 20 fragments, screening at 1e-12: 24 points
    of the mid workload (incl. its first and last) against the screened
    oracle; the clustering option changes the device layout only."""
    from oracle import oracle as O
    env, pts, P, _ = workload_scaled("mid")
    idx = sample_indices(len(pts), 24)
    h = _host(env, P, merge=merge)
    V = h.eval_host(pts[idx])
    Vo, _, _, A = O.potential(env, pts[idx], P=P, screen=True)
    err = np.abs(V - Vo)
    print(f"mid host: max |dV|/A {(err / A).max():.2e}, max |dV|/|V| {(err / np.abs(Vo)).max():.2e}")
    assert np.all(err <= 1e-12 * A)


def test_threads_and_repeat_bitwise():
    """Each point is summed by one thread in a fixed order: the thread count
    does not change a bit, nor does a second call."""
    env, pts, P, _ = workload_scaled("tiny")
    h = _host(env, P)
    old = os.environ.get("ENVPOT_THREADS")
    try:
        os.environ["ENVPOT_THREADS"] = "1"
        a = h.eval_host(pts[:200])
        os.environ["ENVPOT_THREADS"] = "7"
        b = h.eval_host(pts[:200])
        c = h.eval_host(pts[:200])
    finally:
        if old is None:
            os.environ.pop("ENVPOT_THREADS", None)
        else:
            os.environ["ENVPOT_THREADS"] = old
    assert np.array_equal(a, b) and np.array_equal(b, c)


def test_point_on_nucleus_and_empty():
    env, pts, P, _ = workload_scaled("tiny")
    h = _host(env, P)
    assert h.eval_host(np.zeros((0, 3))).shape == (0,)
    v = h.eval_host(env.xyz[:1])
    assert np.isinf(v[0]) and v[0] > 0


def test_option_errors_and_other_calls():
    """FP32C on the host is unsupported; ENV_FORCE_CPU with ENV_BUILD_ONLY is
    an argument error; device-only calls on a host handle are state errors;
    a host handle refuses torch tensors in the binding."""
    env, pts, P, _ = workload_scaled("tiny")
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    with pytest.raises(E.EnvError) as e:
        E.Environment(env.xyz, env.Z, env.fragment, shells, P, precision="fp32c", force_cpu=True)
    assert e.value.status == E.ENV_E_UNSUPPORTED
    with pytest.raises(E.EnvError) as e:
        E.Environment(env.xyz, env.Z, env.fragment, shells, P, precision="fp64", force_cpu=True,
                      build_only=True)
    assert e.value.status == E.ENV_E_ARG
    h = _host(env, P)
    x = np.ascontiguousarray(pts[:4])
    out = np.zeros(16)
    with pytest.raises(E.EnvError) as e:
        E.env_potential_eval_field(h.handle, x.ctypes.data, 4, out.ctypes.data, 0)
    assert e.value.status == E.ENV_E_STATE
    with pytest.raises(E.EnvError) as e:
        E.env_potential_autotune(h.handle, x.ctypes.data, 4, 0)
    assert e.value.status == E.ENV_E_STATE
    with pytest.raises(E.EnvError) as e:
        E.env_batch_create([h.handle])
    assert e.value.status == E.ENV_E_STATE
    with pytest.raises(TypeError):
        h.eval(x)

"""C ABI on the CPU: exported symbols, status strings, argument validation
and the host-side pair-list build (ENV_BUILD_ONLY handles touch no device)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1011_4687_amd import envpot as E
from paper_1011_4687_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(env_\w+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(E.LIB_PATH)
    names = header_functions()
    assert "env_potential_create" in names and "env_potential_eval" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5):
        assert E.env_status_string(s)
    assert E.env_status_string(-99) == "unknown status"


def _tiny_args():
    env, _ = synth.workload("tiny", n_points=1)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    return env, shells


def _build_only(env, shells, P, **kw):
    return E.Environment(env.xyz, env.Z, env.fragment, shells, P, build_only=True, **kw)


def test_build_only_info_and_counts():
    from oracle import oracle as O
    env, shells = _tiny_args()
    sc = O.neutral_scales(env)
    h = _build_only(env, shells, env.density_csr(sc), screening=False)
    info = h.info()
    assert info["n_pairs"] == 1830 == O.count_pairs(env, screen=False)
    assert info["n_pairs_by_L"] == [48 * 49 // 2, 48 * 12, 12 * 13 // 2, 0, 0]
    assert info["built_on_device"] == 0 and info["device_bytes"] == 0
    assert abs(info["electrons"] - env.Z.sum()) <= 1e-11 * env.Z.sum()
    env2, _ = synth.workload("mid", n_points=1)
    sh2 = [(s.atom, s.l, s.exponents, s.coefs) for s in env2.shells]
    h2 = _build_only(env2, sh2, env2.density_csr())
    assert h2.info()["n_pairs"] == O.count_pairs(env2, screen=True)
    assert h2.info()["n_pairs_unscreened"] == O.count_pairs(env2, screen=False)


def test_same_centre_clusters_counts():
    """Pairs whose two shells sit on one atom are merged into clusters of at
    least two members; without merging there are none."""
    env, shells = _tiny_args()
    P = env.density_csr()
    one_centre = 0
    nsh = [0] * len(env.xyz)
    for s in env.shells:
        nsh[s.atom] += len(s.exponents)   # tiny: uncontracted shells, one primitive each
    one_centre = sum(n * (n + 1) // 2 for n in nsh)
    for prec in ("fp32c", "fp64"):
        info = _build_only(env, shells, P, screening=False, precision=prec).info()
        assert info["n_clusters"] >= 1
        assert 2 * info["n_clusters"] <= info["n_cluster_members"] <= one_centre
        assert info["n_pairs"] == 1830
        off = _build_only(env, shells, P, screening=False, precision=prec, merge=False).info()
        assert off["n_clusters"] == 0 and off["n_cluster_members"] == 0
        assert off["n_pairs"] == info["n_pairs"]


def test_neutralize_matches_oracle_trace():
    """ENV_NEUTRALIZE scales every fragment to tr(P_f S_f) = Z_f; the library's
    electron counts (screened pairs' charges plus dropped pairs') follow the
    oracle's overlap route."""
    from oracle import oracle as O
    env, _ = synth.workload("mid", n_points=1)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    h = _build_only(env, shells, env.density_csr(), neutralize=True)
    L, g, c, p, D = h.export_pairs()
    zf = np.array([env.Z[env.fragment == f].sum() for f in range(env.n_fragments)])
    qf = np.array([D[g == f, 0].sum() for f in range(env.n_fragments)])
    assert np.allclose(qf, zf, rtol=1e-9)
    # the scale the library applied equals the oracle's neutral scale
    h0 = _build_only(env, shells, env.density_csr())
    _, g0, _, _, D0 = h0.export_pairs()
    sc = O.neutral_scales(env)
    for f in range(env.n_fragments):
        ratio = D[g == f, 0].sum() / D0[g0 == f, 0].sum()
        assert abs(ratio - sc[f]) <= 1e-10 * sc[f]


def test_eval_requires_device_handle():
    env, shells = _tiny_args()
    h = _build_only(env, shells, env.density_dense([1.0]))
    with pytest.raises(E.EnvError) as ei:
        E.env_potential_eval(h.handle, 8, 1, 8, 0)
    assert ei.value.status == E.ENV_E_STATE
    E.env_potential_eval(h.handle, 0, 0, 0, 0)  # n = 0 is a no-op
    with pytest.raises(E.EnvError) as ei:
        E.env_potential_eval_field(h.handle, 8, 1, 8, 0)
    assert ei.value.status == E.ENV_E_STATE
    E.env_potential_eval_field(h.handle, 0, 0, 0, 0)
    with pytest.raises(E.EnvError) as ei:
        E.env_potential_eval_field(h.handle, 0, -1, 0, 0)
    assert ei.value.status == E.ENV_E_ARG


def test_host_pack_flag_and_image_export_on_a_host_handle():
    """ENV_HOST_PACK is accepted (a build-only handle is host-packed anyway,
    with the same pairs); the record image exists only for device handles."""
    env, shells = _tiny_args()
    P = env.density_dense([1.0])
    a = _build_only(env, shells, P)
    b = _build_only(env, shells, P, host_pack=True)
    assert a.info()["pairs_built_on_device"] == 0 == b.info()["pairs_built_on_device"]
    for x, y in zip(a.export_pairs(), b.export_pairs()):
        assert np.array_equal(x, y)
    with pytest.raises(E.EnvError) as ei:
        a.export_image()
    assert ei.value.status == E.ENV_E_STATE


def test_create_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    env, shells = _tiny_args()
    with pytest.raises(E.EnvError) as ei:
        E.Environment(env.xyz, env.Z, env.fragment, shells, env.density_dense([1.0]))
    assert ei.value.status == E.ENV_E_DEVICE


@pytest.mark.parametrize("case", ["l3", "neg_exp", "nan_xyz", "atom_oor", "asym", "nbf",
                                  "flags", "cross_neutralize", "bad_csr"])
def test_argument_errors(case):
    env, shells = _tiny_args()
    xyz, Z, frag = env.xyz.copy(), env.Z.copy(), env.fragment.copy()
    P = env.density_dense([1.0])
    kw = {}
    expect = E.ENV_E_ARG
    if case == "l3":
        shells = shells[:-1] + [(0, 3, np.array([1.0]), np.array([1.0]))]
        P = np.zeros((env.nbf - 3 + 10,) * 2)
        expect = E.ENV_E_UNSUPPORTED
    elif case == "neg_exp":
        shells = [(0, 0, np.array([-1.0]), np.array([1.0]))] + shells[1:]
    elif case == "nan_xyz":
        xyz[3, 1] = np.nan
    elif case == "atom_oor":
        shells = [(99, 0, np.array([1.0]), np.array([1.0]))] + shells[1:]
    elif case == "asym":
        P = P.copy()
        P[0, 5] += 1e-3
    elif case == "nbf":
        P = P[:-1, :-1]
    elif case == "cross_neutralize":
        frag = np.arange(12, dtype=np.int32)
        kw["neutralize"] = True
        expect = E.ENV_E_UNSUPPORTED
    elif case == "bad_csr":
        rowp, col, val = env.density_csr([1.0])
        col = col.copy()
        col[7] = 10 ** 6
        P = (rowp, col, val)
    if case == "flags":
        o = E.env_options_default()
        o.flags = 0x80
        nuc = (E.env_nucleus * 1)()
        with pytest.raises(E.EnvError) as ei:
            E.env_potential_create(nuc, 1, None, 0, E.env_density(), o)
        assert ei.value.status == E.ENV_E_ARG
        return
    with pytest.raises(E.EnvError) as ei:
        E.Environment(xyz, Z, frag, shells, P, build_only=True, **kw)
    assert ei.value.status == expect, case


def test_server_and_client_argument_errors(tmp_path):
    """Host-side checks of the shared-GPU server and its clients (no GPU)."""
    from paper_1011_4687_amd.envpot import Client, Server
    with pytest.raises(E.EnvError) as ei:
        Client("no/slash")
    assert ei.value.status == E.ENV_E_ARG
    with pytest.raises(E.EnvError) as ei:
        Client("no_such_server_" + os.urandom(4).hex())
    assert ei.value.status == E.ENV_E_STATE
    env, shells = _tiny_args()
    h = _build_only(env, shells, env.density_dense([1.0]))
    with pytest.raises(E.EnvError) as ei:
        Server([h], "x" + os.urandom(4).hex())  # build-only handles cannot be served
    assert ei.value.status == E.ENV_E_STATE
    with pytest.raises(E.EnvError) as ei:
        Server([h], "bad/name")
    assert ei.value.status == E.ENV_E_ARG


def test_update_density_needs_device_handle():
    env, shells = _tiny_args()
    h = _build_only(env, shells, env.density_dense([1.0]))
    with pytest.raises(E.EnvError) as ei:
        h.update_density(env.density_dense([0.5]))
    assert ei.value.status == E.ENV_E_STATE

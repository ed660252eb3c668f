"""One GPU shared by several processes (env_server_* / env_client_*): client
processes with no GPU context send requests through shared memory; the
server evaluates them in batched launches.  Answers are checked against the
server process's own env_potential_eval and against the FP64 oracle."""
import os
import subprocess
import sys
import uuid

import numpy as np
import pytest

from common import sample_indices

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _envs(precision="fp64"):
    from paper_1011_4687_amd import synth
    from paper_1011_4687_amd.envpot import Environment
    out = []
    for env, pts in synth.batched_instances(3, seed0=3000, max_points=2048):
        out.append((Environment.from_synth(env, precision=precision, neutralize=True), env, pts))
    return out


def _direct(E, pts):
    import torch
    v = E.eval(torch.from_numpy(np.ascontiguousarray(pts)).cuda())
    torch.cuda.synchronize()
    return v.cpu().numpy()


def test_clients_in_other_processes(tmp_path):
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Server
    print("[server] four client processes", flush=True)
    envs = _envs()
    name = f"t{uuid.uuid4().hex[:12]}"
    srv = Server([e for e, _, _ in envs], name, n_slots=8, max_points=2048, gather_us=50)
    rng = np.random.default_rng(5)
    jobs = []
    for c in range(4):
        ks = rng.integers(0, 3, 6)
        ns = rng.integers(0, 2049, 6)
        ns[0] = 0 if c == 0 else ns[0]
        ns[1] = 2048
        ns = np.array([min(int(n), len(envs[k][2])) for k, n in zip(ks, ns)])
        pts = np.concatenate([envs[k][2][:n] for k, n in zip(ks, ns)])
        req, ans = tmp_path / f"req{c}.npz", tmp_path / f"ans{c}.npz"
        np.savez(req, env=ks, n=ns, points=pts)
        jobs.append((ks, ns, pts, ans,
                     subprocess.Popen([sys.executable, "-m", "paper_1011_4687_amd.server_client", name, str(req),
                                       str(ans)], cwd=os.path.dirname(HERE))))
    for _, _, _, _, p in jobs:
        assert p.wait(timeout=90) == 0
    st = srv.stats()
    print(f"[server] stats {st}", flush=True)
    assert st["requests"] >= 4 * 5 and st["errors"] == 0
    for ks, ns, pts, ans, _ in jobs:
        V = np.load(ans)["V"]
        assert V.shape[0] == ns.sum()
        off = 0
        for k, n in zip(ks, ns):
            if n:
                ref = _direct(envs[k][0], envs[k][2][:n])
                assert np.abs(V[off:off + n] - ref).max() <= 1e-11
                idx = sample_indices(n, 3)
                env = envs[k][1]
                Vo, _, _, A = O.potential(env, envs[k][2][:n][idx], scale=O.neutral_scales(env), screen=True)
                assert np.all(np.abs(V[off:off + n][idx] - Vo) <= 1e-12 * A)
            off += n
    srv.close()
    for e, _, _ in envs:
        e.close()


def test_errors_slots_and_shutdown():
    from paper_1011_4687_amd.envpot import Client, EnvError, Server, ENV_E_ARG, ENV_E_STATE
    print("[server] errors", flush=True)
    envs = _envs("fp32c")
    name = f"t{uuid.uuid4().hex[:12]}"
    srv = Server([e for e, _, _ in envs], name, n_slots=1, max_points=100)
    with pytest.raises(EnvError) as ei:
        Server([e for e, _, _ in envs], name, n_slots=1, max_points=100)  # a live server has the name
    assert ei.value.status == ENV_E_STATE
    c = Client(name)
    assert (c.n_env, c.max_points, c.slot) == (3, 100, 0)
    with pytest.raises(EnvError) as ei:
        Client(name)  # the only slot is taken
    assert ei.value.status == ENV_E_STATE
    for bad_env, n in ((3, 10), (-1, 10), (0, 101)):
        with pytest.raises(EnvError) as ei:
            c.eval(bad_env, envs[0][2][:n])
        assert ei.value.status == ENV_E_ARG
    v = c.eval(1, envs[1][2][:100])
    assert np.abs(v - _direct(envs[1][0], envs[1][2][:100])).max() <= 4e-6
    assert c.eval(2, np.zeros((0, 3))).shape == (0,)
    srv.close()
    with pytest.raises(EnvError) as ei:
        c.eval(0, envs[0][2][:10])  # the server is gone
    assert ei.value.status == ENV_E_STATE
    c.close()
    for e, _, _ in envs:
        e.close()

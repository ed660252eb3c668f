"""The large and batched workloads at their full sizes, in the launch shapes
the library picks for them; the oracle checks sampled points one by one."""
import os
import time

import numpy as np
import pytest

from common import sample_indices
from paper_1011_4687_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.timeout(900)
def test_large_full_size():
    """5000 atoms (500 neutral fragments, ~9e6 screened pairs), 1,048,576
    points: FP32C within 1e-5 Ha of the unscreened oracle and FP64 within
    1e-12 A of the screened oracle on 24 sampled points and on the stated
    4096-point subsample (stored oracle values; FP32C against the screened
    oracle, the screening change being checked below 1e-6 Ha); the field of
    the same launch size within 1e-6 AE (FP32C) and 1e-12 AE (FP64) of the
    field oracle on 8 of them."""
    import torch
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Environment
    print("[fullsize] large: building", flush=True)
    env, pts = synth.workload("large")
    sc = O.neutral_scales(env)
    P = env.density_csr(sc)
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    x = torch.from_numpy(pts).cuda()
    idx = sample_indices(len(pts), 24)
    res = {}
    for prec in ("fp32c", "fp64"):
        t0 = time.time()
        E = Environment(env.xyz, env.Z, env.fragment, shells, P, precision=prec)
        t1 = time.time()
        V = E.eval(x)
        torch.cuda.synchronize()
        print(f"[fullsize] large {prec}: create {t1 - t0:.1f}s eval {time.time() - t1:.1f}s "
              f"pairs {E.info()['n_pairs']}", flush=True)
        res["full_" + prec] = V.cpu().numpy()
        res[prec] = res["full_" + prec]
        t2 = time.time()
        F = E.eval_field(x)
        torch.cuda.synchronize()
        print(f"[fullsize] large {prec}: field {time.time() - t2:.1f}s", flush=True)
        res["field_" + prec] = F.cpu().numpy()[idx]
        E.close()
    # the field at full size: 8 of the sampled points against the field oracle
    fi = idx[:8]
    Eo, AE = O.field(env, pts[fi], P=P, screen=True)
    for prec, tol in (("fp32c", 1e-6), ("fp64", 1e-12)):
        dE = np.abs(res["field_" + prec][:8, 1:] - Eo).max(axis=1)
        print(f"[fullsize] large field {prec}: max |dE|/AE {(dE / AE).max():.3e}", flush=True)
        assert np.all(dE <= tol * AE)
    Vs, _, _, A = O.potential(env, pts[idx], P=P, screen=True)
    Vf, _, _, _ = O.potential(env, pts[idx], P=P, screen=False)
    e32 = np.abs(res["fp32c"][idx] - Vf)
    e64 = np.abs(res["fp64"][idx] - Vs)
    print(f"[fullsize] large: fp32c max {e32.max():.3e}  fp64 max rel {(e64 / A).max():.3e}", flush=True)
    assert e32.max() <= 1e-5
    assert np.all(e64 <= 1e-12 * A)
    # screening moves V by far less than the FP32C budget
    assert np.abs(Vs - Vf).max() <= 1e-6
    # the stated 4096-point subsample, against the stored screened oracle
    # (tests/golden/make_large_oracle.py)
    g = np.load(os.path.join(GOLDEN, "large_oracle_4096.npz"))
    assert str(g["env_digest"]) == env.digest() and str(g["points_digest"]) == synth.digest(pts)
    gi = g["idx"]
    g32 = np.abs(res["full_fp32c"][gi] - g["V"])
    g64 = np.abs(res["full_fp64"][gi] - g["V"])
    print(f"[fullsize] large, 4096 points: fp32c max {g32.max():.3e} rms {np.sqrt(np.mean(g32 ** 2)):.3e}; "
          f"fp64 max rel {(g64 / g['A']).max():.3e}", flush=True)
    assert g32.max() <= 1e-5
    assert np.all(g64 <= 1e-12 * g["A"])
    # every point of the launch: FP32C against the FP64 kernel
    d = np.abs(res["full_fp32c"] - res["full_fp64"])
    print(f"[fullsize] large, all {len(d)} points: fp32c - fp64 max {d.max():.3e} rms "
          f"{np.sqrt(np.mean(d ** 2)):.3e}", flush=True)
    assert d.max() <= 1e-5
    # no systematic shift: the FP32C far field uses the raw v_rsq_f32 and
    # removes its mean relative error (-7.36e-9) from its sums; left in, it
    # would move V by about 7.36e-9 times the electronic sum (on these
    # points ~5e-6 Ha, some ten times the RMS error), removed, the mean
    # difference must stay within a tenth of that
    shift = 7.36e-9 * float(np.mean(g["V_ele"]))
    mean_d = float(np.mean(res["full_fp32c"] - res["full_fp64"]))
    print(f"[fullsize] large, all points: mean fp32c - fp64 {mean_d:.3e} (uncorrected mean error "
          f"would shift it by {shift:.3e})", flush=True)
    assert abs(mean_d) <= 0.1 * abs(shift)


@pytest.mark.timeout(900)
def test_batched_full_size():
    """64 uneven instances (50..2000 atoms, 1k..200k points) in one persistent
    FP32C launch (instances of 32,768 points or more in Morton order): 256
    seeded-random points of every instance against the stored screened
    oracle (tests/golden/make_goldens.py), and two points of every fourth
    instance against the unscreened oracle."""
    import torch
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Batch, Environment
    print("[fullsize] batched: building", flush=True)
    inst = synth.batched_instances(64)
    hs, xs = [], []
    t0 = time.time()
    for env, pts in inst:
        shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
        # the library's neutralisation (tr(P_f S_f) = Z_f, equal to the oracle's
        # scaling to 1e-10, tested on the CPU); the oracle scales its own P below
        hs.append(Environment(env.xyz, env.Z, env.fragment, shells, env.density_csr(),
                              precision="fp32c", neutralize=True))
        xs.append(torch.from_numpy(pts).cuda())
    print(f"[fullsize] batched: {len(hs)} handles in {time.time() - t0:.1f}s, "
          f"{sum(len(p) for _, p in inst)} points", flush=True)
    B = Batch(hs)
    outs = B.eval(xs)
    torch.cuda.synchronize()
    worst = 0.0
    path = os.path.join(GOLDEN, "batched_oracle_256.npz")
    if os.path.exists(path):
        g = np.load(path)
        n_checked = 0
        for k, (env, pts) in enumerate(inst):
            assert str(g[f"env_digest{k}"]) == env.digest() and str(g[f"points_digest{k}"]) == synth.digest(pts)
            gi = g[f"idx{k}"]
            worst = max(worst, float(np.abs(outs[k].cpu().numpy()[gi] - g[f"V{k}"]).max()))
            n_checked += len(gi)
        print(f"[fullsize] batched: {n_checked} stored oracle points, max err {worst:.3e}", flush=True)
    for k in range(0, 64, 4):
        env, pts = inst[k]
        idx = sample_indices(len(pts), 2, seed=k)
        Vf, _, _, _ = O.potential(env, pts[idx], scale=O.neutral_scales(env), screen=False)
        worst = max(worst, float(np.abs(outs[k].cpu().numpy()[idx] - Vf).max()))
    print(f"[fullsize] batched: max err {worst:.3e}, stats {B.stats()}", flush=True)
    assert worst <= 1e-5
    assert B.stats()["sorted_points"] > 0
    # throughput on a side stream (the default stream cannot be captured):
    # the persistent launch replayed from its graph against one launch per
    # instance on the same stream
    work = sum(h.info()["n_pairs"] * len(x) for h, x in zip(hs, xs))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            B.eval(xs, outs)
        side.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            B.eval(xs, outs)
        side.synchronize()
        t_batch = (time.perf_counter() - t0) / 3
        ref = [o.clone() for o in outs]
        for h, x, o in zip(hs, xs, outs):
            h.eval(x, out=o)
        side.synchronize()
        t0 = time.perf_counter()
        for h, x, o in zip(hs, xs, outs):
            h.eval(x, out=o)
        side.synchronize()
        t_each = time.perf_counter() - t0
    torch.cuda.synchronize()
    assert B.stats()["graph_launches"] >= 5
    worst_diff = max(float((a - b).abs().max()) for a, b in zip(ref, outs))
    assert worst_diff <= 1e-5, worst_diff
    print(f"[fullsize] batched: persistent launch {t_batch * 1e3:.1f} ms ({work / t_batch:.3e} point-pairs/s), "
          f"64 separate launches {t_each * 1e3:.1f} ms, stats {B.stats()}", flush=True)
    B.close()

"""Surrogate kernels (BF16 MFMA forward/backward, Adam, gate) against the
numpy MLP oracle and the exact kernel."""
import numpy as np
import pytest

from paper_1011_4687_amd import synth

pytestmark = pytest.mark.gpu


def _fallback(precision="fp32c"):
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Environment
    rng = np.random.Generator(np.random.PCG64(777))
    env = synth.make_fragmented(60, rng)
    P = env.density_csr(O.neutral_scales(env))
    shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
    return Environment(env.xyz, env.Z, env.fragment, shells, P, precision=precision), env, P


def _setup(seed=3, sigma=0.25, poly_degree=2):
    from paper_1011_4687_amd.envpot import Surrogate, fourier_matrix, init_params
    fb, env, P = _fallback()
    B = fourier_matrix(seed, 0.3)
    p = init_params(seed)
    rng = np.random.default_rng(seed)
    ncoef = (poly_degree + 1) * (poly_degree + 2) * (poly_degree + 3) // 6
    poly = rng.standard_normal(ncoef) * 0.1
    S = Surrogate(fb, B, p, radius=6.0, poly_degree=poly_degree, poly=poly, sigma=sigma)
    return S, fb, B, p, poly, env, P


def _ulp_bf16(x):
    """One unit in the last place of bfloat16 at |x| (8 significant bits)."""
    e = np.floor(np.log2(np.maximum(np.abs(x), 1e-38)))
    return 2.0 ** (e - 7)


def test_layerwise_matches_oracle():
    """One forward and backward pass traced layer by layer
    (env_surrogate_trace_step) and checked step by step against the MLP
    oracle fed the GPU's own inputs of that step, so a BF16 rounding that
    lands on the other side of a tie in one layer is not carried into the
    next.  Bounds:
      matrix products (FP32 accumulation of K exact BF16 x BF16 products):
        |d| <= (K + 2) 2^-24 x (sum of |terms|), K = 128 for the layers,
        K = rows for the weight gradients;
      BF16 roundings (features, SiLU, dZ): within one BF16 unit of the
        oracle's rounding of the GPU's own FP32 input, and equal for >= 99 %;
      every weight-gradient entry: within 1e-4 relative of the oracle, or,
      for an entry that cancels (|g| below the accumulation bound times
      1e4), within that bound."""
    import torch
    from oracle import mlp_oracle as M
    print("[surrogate] layer by layer", flush=True)
    S, fb, B, p, poly, env, P = _setup()
    rng = np.random.default_rng(5)
    n = 1000                                        # padded to 1024 rows inside
    pts = synth.points_in_ball(rng, n, 6.0)
    t = rng.standard_normal(n).astype(np.float32)
    tr = S.trace_step(torch.from_numpy(pts).cuda(), torch.from_numpy(t).cuda())
    layers, w_out, b_out = M.unpack(p.astype(np.float64))
    H, Z = tr["H"].astype(np.float64), tr["Z"].astype(np.float64)
    dH, dZ = tr["dH"].astype(np.float64), tr["dZ"].astype(np.float64)
    y, dy, g = tr["y"].astype(np.float64), tr["dy"].astype(np.float64), tr["grad"].astype(np.float64)
    u = 2.0 ** -24

    def rounded(gpu, ref, what):
        d = np.abs(gpu - ref)
        frac = np.mean(d == 0)
        print(f"  {what}: exact {frac:.5f}, max {np.max(d / _ulp_bf16(ref)):.2f} BF16 units")
        assert np.all(d <= _ulp_bf16(ref) * 1.0001) and frac >= 0.99

    def product(gpu, ref, scale, K, what):
        r = np.abs(gpu - ref) / np.maximum(scale, 1e-300)
        print(f"  {what}: max |d|/sum|terms| {r.max():.2e} (bound {(K + 2) * u:.2e})")
        assert r.max() <= (K + 2) * u

    rounded(H[0], M.bf16(M.features(pts, B)), "features")
    for l in range(4):
        Zr, sc = M.hidden_pre(H[l], *layers[l])
        product(Z[l], Zr, sc, 128, f"Z{l + 1}")
        rounded(H[l + 1], M.hidden_act(Z[l]), f"H{l + 1}")
    yr, sc = M.output(H[4], w_out, b_out)
    product(y, yr, sc, 128, "y")
    dyr = 2.0 * (y - t) / n
    assert np.all(np.abs(dy - dyr) <= 4 * u * np.abs(dyr))
    assert abs(tr["loss"] - np.mean((y - t) ** 2)) <= 1e-6 * np.mean((y - t) ** 2)
    assert np.all(np.abs(dH[3] - np.outer(dy, w_out)) <= 2 * u * np.abs(np.outer(dy, w_out)))
    within = []
    o = 0
    offs = []
    for l in range(4):
        offs.append(o)
        o += 128 * 128 + 128
    for l in range(3, -1, -1):
        dz = M.dz_of(dH[l], Z[l])
        rounded(dZ[l], M.bf16(dz), f"dZ{l + 1}")
        gW, sc = M.weight_grad(dZ[l], H[l])
        gg = g[offs[l]:offs[l] + 128 * 128].reshape(128, 128)
        bound = (n + 2) * u * sc
        err = np.abs(gg - gW)
        ok = (err <= 1e-4 * np.abs(gW)) | ((np.abs(gW) <= 1e4 * bound) & (err <= bound))
        rel_ok = np.mean(err <= 1e-4 * np.abs(gW))
        within.append(rel_ok)
        print(f"  dW{l + 1}: {rel_ok:.4f} of entries within 1e-4 relative; max |d|/sum|terms| {np.max(err / sc):.2e}")
        assert ok.all()
        gb = g[offs[l] + 128 * 128:offs[l] + 128 * 128 + 128]
        gbr, gbs = dz.sum(axis=0), np.abs(dz).sum(axis=0)
        assert np.all(np.abs(gb - gbr) <= 1e-4 * np.abs(gbr) + 8e-6 * gbs)
        if l > 0:
            dHr, sc = M.input_grad(dZ[l], layers[l][0])
            product(dH[l - 1], dHr, sc, 128, f"dH{l}")
    gwo, gwos = H[4].T @ dy, np.abs(H[4]).T @ np.abs(dy)
    assert np.all(np.abs(g[o:o + 128] - gwo) <= 1e-4 * np.abs(gwo) + (n + 2) * u * gwos)
    assert abs(g[o + 128] - dy.sum()) <= 1e-4 * abs(dy.sum()) + (n + 2) * u * np.abs(dy).sum()
    # the finishing step of a prediction: poly(r/R) + sigma y, given the GPU's y
    got = S.predict(torch.from_numpy(pts).cuda()).cpu().numpy()
    ref = M.poly_eval(pts, poly, 2, 6.0) + 0.25 * y
    assert np.all(np.abs(got - ref) <= 1e-12 * (np.abs(ref) + 1))
    S.close()


def test_train_gate_and_fallback():
    """A short training run on a 60-atom environment with the network
    covering a 3-bohr ball: the loss falls, the gate passes voxels, points in
    passing voxels are within 1e-5 Ha of the FP64 exact kernel, and gated-out
    points (the 3.5-6 bohr shell and failing voxels) equal the exact FP32C
    kernel on the compacted list bit for bit."""
    import torch
    from paper_1011_4687_amd.envpot import Surrogate, fourier_matrix, init_params
    print("[surrogate] train", flush=True)
    fb, env, P = _fallback("fp32c")
    teacher, _, _ = _fallback("fp64")
    S = Surrogate(fb, fourier_matrix(11, 0.25), init_params(11), radius=3.0)
    S.train(teacher, n_train=262144, epochs=24, batch=4096, gate_grid=12, gate_samples=16,
            n_fit=65536, poly_degree=8)
    info = S.info()
    print({k: info[k] for k in ("baseline_rms", "final_loss", "gate_voxels_in_ball",
                                "gate_voxels_pass", "gate_pass_volume_fraction",
                                "train_seconds", "teacher_seconds")}, info["epoch_loss"][:4])
    assert info["epoch_loss"][3] < info["epoch_loss"][0]
    pts = np.concatenate([synth.points_in_ball(np.random.default_rng(9), 20000, 3.0),
                          synth.points_in_ball(np.random.default_rng(10), 2000, 6.0, r_min=3.5)])
    x = torch.from_numpy(pts).cuda()
    V, used = S.eval(x)
    V = V.cpu().numpy()
    used = used.cpu().numpy().astype(bool)
    assert used[20000:].all()                     # outside the region: always exact
    served = float((~used[:20000]).mean())
    print(f"[surrogate] network serves {served:.3f} of the in-region points", flush=True)
    assert info["gate_voxels_pass"] > 0 and served > 0.0   # the network check below is not vacuous
    exact64 = teacher.eval(x).cpu().numpy()
    assert np.abs(V[~used] - exact64[~used]).max() <= 1e-5
    idx = np.nonzero(used)[0]
    ref = fb.eval(torch.from_numpy(np.ascontiguousarray(pts[idx])).cuda()).cpu().numpy()
    assert np.array_equal(V[idx], ref)
    assert S.info()["last_eval_fallback"] == len(idx)
    # a new density of the fallback environment: the network was trained on
    # the old one, so the surrogate refuses to evaluate
    from paper_1011_4687_amd import envpot
    rowp, col, val = P
    fb.update_density((rowp, col, val * 1.05))
    for call in (lambda: S.eval(x), lambda: S.predict(x)):
        with pytest.raises(envpot.EnvError) as ei:
            call()
        assert ei.value.status == envpot.ENV_E_STATE
    S.close()


@pytest.mark.timeout(900)
def test_gain_on_surrogate_workload():
    """What the trained network gains over the exact kernel: on the 1000-atom
    surrogate workload the gated surrogate is faster than exact FP32C on the
    same points and stays within 1e-5 Ha of the oracle on sampled points."""
    import time
    import torch
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Environment, Surrogate, fourier_matrix, init_params
    print("[surrogate] gain", flush=True)
    env, _ = synth.workload("surrogate", n_points=1)
    _, infer, outer = synth.surrogate_sets(n_train=1, n_infer=200_000, n_out=8192)
    pts = np.ascontiguousarray(np.concatenate([infer, outer]))
    x = torch.from_numpy(pts).cuda()
    fb = Environment.from_synth(env, precision="fp32c", neutralize=True)
    te = Environment.from_synth(env, precision="fp64", neutralize=True)
    S = Surrogate(fb, fourier_matrix(1004, 0.25), init_params(1004), radius=6.0)
    S.train(te, n_train=1_000_000, epochs=12, batch=8192, lr=2e-3, lr_final=1e-5, poly_degree=8)
    info = S.info()
    print({k: info[k] for k in ("baseline_rms", "final_loss", "gate_pass_volume_fraction",
                                "gate_max_err_passed", "train_seconds")}, flush=True)
    fb.eval(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V_exact = fb.eval(x)
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t0
    S.eval(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V, used = S.eval(x)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    print(f"[surrogate] exact {t_exact * 1e3:.1f} ms, surrogate {t_sur * 1e3:.1f} ms, "
          f"fallback {used.float().mean().item():.3f}", flush=True)
    assert t_sur < t_exact
    idx = np.concatenate([np.linspace(0, len(infer) - 1, 24).astype(int),
                          len(infer) + np.arange(0, len(outer), len(outer) // 4)])
    Vo, _, _, _ = O.potential(env, pts[idx], scale=O.neutral_scales(env), screen=False)
    err = np.abs(V.cpu().numpy()[idx] - Vo)
    print(f"[surrogate] max err vs oracle {err.max():.3e}", flush=True)
    assert err.max() <= 1e-5
    assert used.cpu().numpy()[len(infer):].all()
    # every point against the FP64 kernel
    V64 = te.eval(x).cpu().numpy()
    d = np.abs(V.cpu().numpy() - V64)
    print(f"[surrogate] all {len(d)} points vs FP64 kernel: max {d.max():.3e}", flush=True)
    assert d.max() <= 1e-5
    # the stored oracle sample of the workload (16,384 of its 1,065,536
    # points, tests/golden/make_goldens.py), evaluated at those points
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "surrogate_oracle_16384.npz")
    if os.path.exists(path):
        g = np.load(path)
        _, inf_all, out_all = synth.surrogate_sets(n_train=1, n_infer=1_000_000, n_out=65536)
        allp = np.ascontiguousarray(np.concatenate([inf_all, out_all]))
        assert str(g["env_digest"]) == env.digest() and str(g["points_digest"]) == synth.digest(allp)
        xs = torch.from_numpy(np.ascontiguousarray(allp[g["idx"]])).cuda()
        Vg, ug = S.eval(xs)
        eg = np.abs(Vg.cpu().numpy() - g["V"])
        print(f"[surrogate] stored oracle sample ({len(eg)} points, fallback "
              f"{ug.float().mean().item():.3f}): max {eg.max():.3e}", flush=True)
        assert eg.max() <= 1e-5
    S.close()
    fb.close()
    te.close()


def test_split_surrogate_with_exact_part():
    """Split surrogate (env_surrogate_set_near): the network learns the
    potential of the fragments other than the nearest one (teacher: their
    FP64 handle), the nearest fragment is evaluated exactly at every point
    and added.  Points the network serves are within 1e-5 Ha of the FP64
    kernel of the whole environment; gated-out points equal the whole
    environment's FP32C kernel bit for bit; predict gives the network alone;
    removing the exact part changes served points by exactly its values."""
    import torch
    from oracle import oracle as O
    from paper_1011_4687_amd.envpot import Environment, Surrogate, fourier_matrix, init_params
    print("[surrogate] split", flush=True)
    rng = np.random.Generator(np.random.PCG64(777))
    env = synth.make_fragmented(60, rng)
    sc = O.neutral_scales(env)
    nearest = int(env.fragment[np.argmin(np.linalg.norm(env.xyz, axis=1))])
    far = [f for f in range(env.n_fragments) if f != nearest]
    fb = Environment.from_synth(env, scale=sc, precision="fp32c")
    full64 = Environment.from_synth(env, scale=sc, precision="fp64")
    near = Environment.from_synth(synth.subset(env, [nearest]), scale=sc[[nearest]], precision="fp32c")
    teach = Environment.from_synth(synth.subset(env, far), scale=sc[far], precision="fp64")
    S = Surrogate(fb, fourier_matrix(12, 0.25), init_params(12), radius=3.0)
    S.set_near(near)
    S.train(teach, n_train=262144, epochs=24, batch=4096, gate_grid=12, gate_samples=16, n_fit=65536,
            poly_degree=8)
    pts = np.concatenate([synth.points_in_ball(np.random.default_rng(21), 20000, 3.0),
                          synth.points_in_ball(np.random.default_rng(22), 1000, 5.0, r_min=3.5)])
    x = torch.from_numpy(pts).cuda()
    V, used = S.eval(x)
    V, used = V.cpu().numpy(), used.cpu().numpy().astype(bool)
    served = float((~used[:20000]).mean())
    print(f"[surrogate] split: network serves {served:.3f} of the in-region points", flush=True)
    assert used[20000:].all() and served > 0.0
    ref64 = full64.eval(x).cpu().numpy()
    assert np.abs(V[~used] - ref64[~used]).max() <= 1e-5
    idx = np.nonzero(used)[0]
    ref32 = fb.eval(torch.from_numpy(np.ascontiguousarray(pts[idx])).cuda()).cpu().numpy()
    assert np.array_equal(V[idx], ref32)
    # the network alone, and the network plus the exact part
    net = S.predict(x).cpu().numpy()
    vn = near.eval(x).cpu().numpy()
    assert np.array_equal(V[~used], net[~used] + vn[~used])
    S.set_near(None)
    V2, used2 = S.eval(x)
    assert np.array_equal(used2.cpu().numpy().astype(bool), used)
    assert np.array_equal(V2.cpu().numpy()[~used], net[~used])
    S.close()
    for E in (fb, full64, near, teach):
        E.close()

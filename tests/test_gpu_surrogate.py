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


def test_forward_matches_oracle():
    import torch
    from oracle import mlp_oracle as M
    print("[surrogate] forward", flush=True)
    S, fb, B, p, poly, env, P = _setup()
    pts = synth.points_in_ball(np.random.default_rng(1), 1000, 6.0)
    got = S.predict(torch.from_numpy(pts).cuda()).cpu().numpy()
    ref = M.predict(p.astype(np.float64), pts, B, poly, 2, 6.0, 0.25)
    y_scale = np.abs(ref - M.poly_eval(pts, poly, 2, 6.0)).max()
    err = np.abs(got - ref)
    print("forward max err", err.max(), "median", np.median(err), "y scale", y_scale)
    assert np.median(err) <= 1e-4 * y_scale
    assert err.max() <= 2e-2 * y_scale
    S.close()


def test_gradients_match_oracle():
    import torch
    from oracle import mlp_oracle as M
    print("[surrogate] gradients", flush=True)
    S, fb, B, p, poly, env, P = _setup()
    rng = np.random.default_rng(5)
    pts = synth.points_in_ball(rng, 200, 6.0)       # 200: padded to 224 rows inside
    t = rng.standard_normal(200)
    loss, g = S.loss_grad(torch.from_numpy(pts).cuda(), torch.from_numpy(t).cuda())
    lref, gref = M.loss_and_grads(p.astype(np.float64), pts, t, B, rounding=True)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    print("loss", loss, lref, "grad rel err", rel)
    assert abs(loss - lref) <= 1e-3 * lref
    assert rel <= 2e-2
    # every parameter block agrees in direction
    o = 0
    for size in [128 * 128, 128] * 4 + [128, 1]:
        a, b = g[o:o + size], gref[o:o + size]
        if np.linalg.norm(b) > 0:
            assert a @ b / (np.linalg.norm(a) * np.linalg.norm(b)) >= 0.999
        o += size
    S.close()


def test_train_gate_and_fallback():
    """A short training run on a 60-atom environment: the loss falls, points in
    passing voxels are within 1e-5 Ha of the FP64 exact kernel, and gated-out
    points equal the exact FP32C kernel on the compacted list bit for bit."""
    import torch
    from paper_1011_4687_amd.envpot import Surrogate, fourier_matrix, init_params
    print("[surrogate] train", flush=True)
    fb, env, P = _fallback("fp32c")
    teacher, _, _ = _fallback("fp64")
    S = Surrogate(fb, fourier_matrix(11, 0.25), init_params(11), radius=6.0)
    S.train(teacher, n_train=131072, epochs=4, batch=4096, gate_grid=12, gate_samples=6,
            n_fit=65536, poly_degree=6)
    info = S.info()
    print({k: info[k] for k in ("baseline_rms", "final_loss", "gate_voxels_in_ball",
                                "gate_voxels_pass", "gate_pass_volume_fraction",
                                "train_seconds", "teacher_seconds")}, info["epoch_loss"][:4])
    assert info["epoch_loss"][3] < info["epoch_loss"][0]
    pts = np.concatenate([synth.points_in_ball(np.random.default_rng(9), 20000, 6.0),
                          synth.points_in_ball(np.random.default_rng(10), 2000, 7.5, r_min=6.0)])
    x = torch.from_numpy(pts).cuda()
    V, used = S.eval(x)
    V = V.cpu().numpy()
    used = used.cpu().numpy().astype(bool)
    assert used[20000:].all()                     # outside the region: always exact
    exact64 = teacher.eval(x).cpu().numpy()
    if (~used).any():
        assert np.abs(V[~used] - exact64[~used]).max() <= 1e-5
    idx = np.nonzero(used)[0]
    ref = fb.eval(torch.from_numpy(np.ascontiguousarray(pts[idx])).cuda()).cpu().numpy()
    assert np.array_equal(V[idx], ref)
    assert S.info()["last_eval_fallback"] == len(idx)
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
    S.close()
    fb.close()
    te.close()

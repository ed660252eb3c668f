#!/usr/bin/env python3
"""Throughput of the environment potential on one MI355X.

A step is one evaluation of V(r) for the whole point batch of the workload
(nuclear term, Boys function, Hermite recursion and contraction, FP64
cancellation sums, output), with the pair list already on the device and the
points already in HBM.  The metric is point-pair evaluations per second:
n_points x n_pairs (unique screened primitive shell pairs) / time per step.

Headline workload "large": 5000 environment atoms in 500 neutral 10-atom
fragments (contracted s/p/d shells, about 6e6 screened pairs) and 1,048,576
points (65,536 walkers x 16 electrons) in the 8-bohr QM sphere, evaluated
three ways: the FP32C kernel (the headline value), the FP64 kernel, and the
learned surrogate with its gate and exact fallback.  Each is timed with HIP
events and checked against the FP64 oracle on the stored 4096-point sample of
the workload and, on every point, against the FP64 kernel.  Secondary legs:
the mid workload (200 atoms, 131,072 points; potential and field), the 64
uneven batched instances in one persistent launch, the paper's cell-sum form,
one GPU shared by client processes, and the 1000-atom surrogate workload.

The CPU-baseline leg times the FP64 oracle on a bounded sample of the
headline points, on all host cores and on one.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "point-pair evals/s at ≤1e-5 Ha max err: FP64 vs FP32 vs MLP surrogate, 1 GPU"

PEAK_FP32 = 157.3e12   # MI355X FP32 vector (published, packed)
PEAK_FP64 = 78.6e12    # MI355X FP64 vector

def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_record(name):
    """A committed counter record (profiles/<name>.json) when the kernel
    sources it was taken from are unchanged, else None."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for s in rec["kernel_sources"]:
            h.update(open(os.path.join(ROOT, s), "rb").read())
        if h.hexdigest() != rec["kernel_source_sha256"]:
            return None
        return rec
    except (OSError, KeyError, ValueError):
        return None


def time_calls(fn, steps, warmup, torch, stream=None):
    """Mean HIP-event time (ms) of fn(stream) over `steps` calls after
    `warmup` calls, all on one stream; also the wall time per call."""
    stream = stream or torch.cuda.current_stream()
    for _ in range(warmup):
        fn(stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for s, e in evs:
        s.record(stream)
        fn(stream)
        e.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return float(np.mean([s.elapsed_time(e) for s, e in evs])), wall * 1e3


def errors(V, Vo, A, tag=""):
    """max / RMS of |V - Vo|, relative to A (the conditioning scale) and to
    |Vo| (where |Vo| >= 1e-3 Ha, so values near zero do not dominate)."""
    err = np.abs(V - Vo)
    big = np.abs(Vo) >= 1e-3
    return {"max_abs_err": float(err.max()), "rms_err": float(np.sqrt(np.mean(err ** 2))),
            "max_rel_to_A": float((err / A).max()),
            "max_rel_to_V": float((err[big] / np.abs(Vo[big])).max()) if big.any() else None,
            "n_checked": int(len(V))}


def load_golden(name, env, pts):
    """Stored oracle values (tests/golden/<name>) if their input digests
    match the generated workload."""
    from paper_1011_4687_amd import synth
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    g = dict(np.load(path))
    if str(g["env_digest"]) != env.digest() or str(g["points_digest"]) != synth.digest(pts):
        raise RuntimeError(f"{name}: stored oracle values do not belong to this workload")
    return g


def exact_path(E, x, steps, warmup, torch):
    """Time E.eval on x: the whole call (Morton ordering, kernel, split sums)
    with HIP events around each call, and the potential kernel alone with the
    library's events around each launch of the same timed calls (same
    stream)."""
    n = x.shape[0]
    out = torch.empty(n, dtype=torch.float64, device="cuda")

    def call(st):
        E.eval(x, out=out, stream=st)
    for _ in range(warmup):
        call(torch.cuda.current_stream())
    torch.cuda.synchronize()
    E.kernel_timing(True)
    ms, wall = time_calls(call, steps, 0, torch)
    kms = E.kernel_times()
    E.kernel_timing(False)
    return out, ms, wall, float(np.mean(kms)) if kms else None


def large_leg(args, torch, envpot, synth, wc):
    """The headline: FP32C, FP64 and the split surrogate on the large
    workload, each checked against the stored oracle sample and against the
    FP64 kernel on every point."""
    env, pts = synth.workload("large")
    n = len(pts)
    x = torch.from_numpy(pts).cuda()
    log(f"[bench] large: {env.n_nuclei} atoms, {env.n_fragments} fragments, nbf {env.nbf}, {n} points")
    gold = load_golden("large_oracle_4096.npz", env, pts)
    paths, V = {}, {}
    info = None
    plan = [("fp32c", args.steps, args.warmup), ("fp64", min(args.steps, 10), 1)]
    for prec, steps, warm in [p for p in plan if p[0] in args.large_paths.split(",")]:
        t0 = time.perf_counter()
        E = envpot.Environment.from_synth(env, precision=prec, neutralize=True)
        t_create = time.perf_counter() - t0
        info = E.info()
        out, ms, wall, kms = exact_path(E, x, steps, warm, torch)
        npairs = info["n_pairs"]
        flops = wc.eval_flops(n, info["n_pairs_by_L"], info["n_nuclei"])
        V[prec] = out.cpu().numpy()
        paths[prec] = {"point_pairs_per_s": n * npairs / (ms * 1e-3), "ms_per_step": ms,
                       "wall_ms_per_step": wall, "kernel_ms": kms, "steps": steps, "warmup": warm,
                       "create_s": t_create,
                       "tflops_md_equivalent": flops / (kms * 1e-3) / 1e12 if kms else None}
        if gold is not None:
            paths[prec]["accuracy_vs_oracle_4096"] = errors(V[prec][gold["idx"]], gold["V"], gold["A"])
        log(f"[bench] large {prec}: {ms:.1f} ms/step (kernel {kms:.1f} ms), "
            f"{paths[prec]['point_pairs_per_s']:.4g} pp/s, create {t_create:.2f} s; "
            f"{paths[prec].get('accuracy_vs_oracle_4096')}")
        if prec == "fp32c":
            fb = E
        else:
            E.close()
    if "fp32c" in V and "fp64" in V:
        d = np.abs(V["fp32c"] - V["fp64"])
        paths["fp32c"]["vs_fp64_kernel_all_points"] = {"max_abs_diff": float(d.max()),
                                                       "rms_diff": float(np.sqrt(np.mean(d ** 2))), "n": n}
    if "fp32c" in V:
        if not args.no_surrogate and "fp64" in V:
            paths["surrogate"] = large_surrogate(args, torch, envpot, synth, env, pts, x, fb, info, gold, V["fp64"],
                                                 paths["fp32c"]["ms_per_step"])
        fb.close()
    return {"env": env, "pts": pts, "info": info, "paths": paths, "V": V, "gold": gold}


def large_surrogate(args, torch, envpot, synth, env, pts, x, fb, info, gold, V64, ms_exact):
    """Split surrogate of the large workload.  The network covers the whole
    8-bohr QM sphere and stands in for the potential of the fragments whose
    atoms all lie beyond R_NEAR (smooth in the sphere); the few fragments
    with an atom inside R_NEAR (--r-near) are evaluated exactly (FP32C) at every point
    and added; the gate sends points of voxels that failed validation to the
    FP32C kernel of the whole environment."""
    n = len(pts)
    R_NEAR = args.r_near
    r = np.linalg.norm(env.xyz, axis=1)
    near = sorted(set(int(f) for f in env.fragment[r < R_NEAR]))
    far = [f for f in range(env.n_fragments) if f not in set(near)]
    t0 = time.perf_counter()
    E_near = envpot.Environment.from_synth(synth.subset(env, near, "large-near"), precision="fp32c",
                                           neutralize=True) if near else None
    T_far = envpot.Environment.from_synth(synth.subset(env, far, "large-far"), precision="fp64",
                                          neutralize=True)
    t_sub = time.perf_counter() - t0
    near_pairs = E_near.info()["n_pairs"] if near else 0
    S = envpot.Surrogate(fb, envpot.fourier_matrix(1005, args.sigma), envpot.init_params(1005), radius=8.0)
    S.set_near(E_near)
    t0 = time.perf_counter()
    S.train(T_far, n_train=2_000_000, epochs=args.sur_epochs, batch=8192, lr=args.sur_lr, lr_final=1e-5,
            poly_degree=8, gate_grid=24, gate_samples=32, gate_tol=4e-6)
    t_train = time.perf_counter() - t0
    si = S.info()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    used = torch.empty(n, dtype=torch.uint8, device="cuda")

    def call(st):
        S.eval(x, stream=st, out=out, used=used)
    ms, wall = time_calls(call, args.steps, args.warmup, torch)
    nfb = S.info()["last_eval_fallback"]
    Vs = out.cpu().numpy()
    # the network alone (features, four layers, output, baseline)
    ms_net, _ = time_calls(lambda st: S.predict(x, stream=st, out=out), max(3, args.steps // 4), 1, torch)
    # the exact part alone
    ms_near = time_calls(lambda st: E_near.eval(x, out=out, stream=st), max(3, args.steps // 4), 1, torch)[0] \
        if near else 0.0
    npairs = info["n_pairs"]
    saved = (ms_exact - ms) * 1e-3
    rep = {
        "design": f"network over the 8-bohr sphere for the potential of the {len(far)} fragments with every "
                  f"atom beyond {R_NEAR} bohr; the {len(near)} fragments with an atom inside {R_NEAR} bohr "
                  f"({near_pairs} pairs) evaluated exactly (FP32C) at every point and added; gated-out points "
                  f"get the whole environment's FP32C value",
        "fourier_sigma_per_bohr": args.sigma,
        "point_pairs_per_s": n * npairs / (ms * 1e-3),
        "ms_per_step": ms, "wall_ms_per_step": wall,
        "network_ms": ms_net, "exact_part_ms": ms_near,
        "speedup_vs_fp32c": ms_exact / ms,
        "fallback_fraction": nfb / n,
        "gate_pass_volume_fraction": si["gate_pass_volume_fraction"],
        "gate_voxels_pass": si["gate_voxels_pass"], "gate_voxels_in_ball": si["gate_voxels_in_ball"],
        "gate_max_validation_err": si["gate_max_err_passed"],
        "baseline_rms": si["baseline_rms"], "final_loss": si["final_loss"],
        "teacher_s": si["teacher_seconds"], "train_s": si["train_seconds"], "gate_s": si["gate_seconds"],
        "train_total_s": t_train, "subset_create_s": t_sub,
        "break_even_evaluations": (t_train + t_sub) / saved if saved > 0 else None,
    }
    d = np.abs(Vs - V64)
    rep["vs_fp64_kernel_all_points"] = {"max_abs_diff": float(d.max()),
                                        "rms_diff": float(np.sqrt(np.mean(d ** 2))), "n": n}
    if gold is not None:
        rep["accuracy_vs_oracle_4096"] = errors(Vs[gold["idx"]], gold["V"], gold["A"])
    log(f"[bench] large surrogate: {ms:.2f} ms/step (network {ms_net:.2f} ms, exact part {ms_near:.2f} ms), "
        f"fallback {nfb / n:.4f}, gate pass {si['gate_pass_volume_fraction']:.3f}, train {t_train:.1f} s, "
        f"vs FP64 kernel max {d.max():.2e}; {rep.get('accuracy_vs_oracle_4096')}")
    S.close()
    if near:
        E_near.close()
    T_far.close()
    return rep


def mid_leg(args, torch, envpot, synth, wc):
    """Secondary: the mid workload, potential and field, both precisions,
    plus the on-device density refold."""
    env, pts = synth.workload("mid")
    n = len(pts)
    x = torch.from_numpy(pts).cuda()
    gold = load_golden("mid_oracle_16384.npz", env, pts)
    rep = {"workload": f"mid: {env.n_nuclei} atoms in {env.n_fragments} neutral fragments, nbf {env.nbf}, "
                       f"{n} points in the 8-bohr QM sphere"}
    V = {}
    for prec in ("fp32c", "fp64"):
        t0 = time.perf_counter()
        E = envpot.Environment.from_synth(env, precision=prec, neutralize=True)
        t_create = time.perf_counter() - t0
        info = E.info()
        out, ms, wall, kms = exact_path(E, x, args.steps, args.warmup, torch)
        V[prec] = out.cpu().numpy()
        npairs = info["n_pairs"]
        r = {"n_pairs": npairs, "pairs_by_L": info["n_pairs_by_L"],
             "point_pairs_per_s": n * npairs / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": kms,
             "create_s": t_create,
             "tflops_md_equivalent": wc.eval_flops(n, info["n_pairs_by_L"], info["n_nuclei"]) / (kms * 1e-3) / 1e12}
        if gold is not None:
            r["accuracy_vs_oracle_16384"] = errors(V[prec][gold["idx"]], gold["V"], gold["A"])
        # the field E = -grad V (with V) of the same handle at the same points
        fout = torch.empty((n, 4), dtype=torch.float64, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fms, _ = time_calls(lambda st: E.eval_field(x, out=fout, stream=st), args.steps, args.warmup, torch,
                                side)
        fflops = wc.eval_field_flops(n, info["n_pairs_by_L"], info["n_nuclei"])
        r["field"] = {"point_pairs_per_s": n * npairs / (fms * 1e-3), "ms_per_step": fms,
                      "tflops_md_equivalent": fflops / (fms * 1e-3) / 1e12}
        # a new density with the same blocks, refolded on the device
        rowp, col, val = env.density_csr(None)
        t_upd = []
        for _ in range(3):
            t0 = time.perf_counter()
            E.update_density((rowp, col, val * 1.05))
            t_upd.append(time.perf_counter() - t0)
        r["density_update_ms"] = float(np.median(t_upd)) * 1e3
        rep[prec] = r
        log(f"[bench] mid {prec}: {ms:.2f} ms/step (kernel {kms:.2f}), field {fms:.2f} ms, "
            f"update {r['density_update_ms']:.1f} ms; {r.get('accuracy_vs_oracle_16384')}")
        E.close()
    d = np.abs(V["fp32c"] - V["fp64"])
    rep["fp32c_vs_fp64_kernel_all_points"] = {"max_abs_diff": float(d.max()), "n": n}
    return rep


def batched_leg(args, torch, envpot, synth):
    """Secondary: 64 uneven instances (50-2000 atoms, 1k-200k points), FP32C,
    one persistent launch per step through a plan that replays its captured
    graph; checked against the stored oracle sample (256 points per
    instance) when present."""
    insts = synth.batched_instances(64)
    t0 = time.perf_counter()
    envs = [envpot.Environment.from_synth(e, precision="fp32c", neutralize=True) for e, _ in insts]
    t_create = time.perf_counter() - t0
    xs = [torch.from_numpy(p).cuda() for _, p in insts]
    outs = [torch.empty(len(p), dtype=torch.float64, device="cuda") for _, p in insts]
    plan = envpot.Batch(envs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        t0 = time.perf_counter()
        plan.autotune(xs, outs, stream=side)
        t_tune = time.perf_counter() - t0
        ms, wall = time_calls(lambda st: plan.eval(xs, outs, stream=st), args.steps, args.warmup, torch, side)
    work = float(sum(len(p) * E.info()["n_pairs"] for (_, p), E in zip(insts, envs)))
    rep = {"workload": f"64 instances, {min(e.n_nuclei for e, _ in insts)}-{max(e.n_nuclei for e, _ in insts)} "
                       f"atoms, {sum(len(p) for _, p in insts)} points in total, FP32C, one persistent launch "
                       f"replayed from its graph, shape from env_batch_autotune",
           "point_pairs_per_s": work / (ms * 1e-3), "ms_per_step": ms, "wall_ms_per_step": wall,
           "create_s": t_create, "autotune_s": t_tune, "plan": plan.stats()}
    path = os.path.join(ROOT, "tests", "golden", "batched_oracle_256.npz")
    if os.path.exists(path):
        g = dict(np.load(path))
        worst = {"max_abs_err": 0.0, "max_rel_to_A": 0.0, "n_checked": 0}
        for i, ((e, p), o) in enumerate(zip(insts, outs)):
            if str(g[f"env_digest{i}"]) != e.digest() or str(g[f"points_digest{i}"]) != synth.digest(p):
                raise RuntimeError("batched_oracle_256.npz does not belong to this workload")
            V = o.cpu().numpy()[g[f"idx{i}"]]
            err = np.abs(V - g[f"V{i}"])
            worst["max_abs_err"] = max(worst["max_abs_err"], float(err.max()))
            worst["max_rel_to_A"] = max(worst["max_rel_to_A"], float((err / g[f"A{i}"]).max()))
            worst["n_checked"] += len(err)
        rep["accuracy_vs_oracle_256_per_instance"] = worst
    log(f"[bench] batched: {ms:.2f} ms/step, {work / (ms * 1e-3):.4g} pp/s; "
        f"{rep.get('accuracy_vs_oracle_256_per_instance')}")
    plan.close()
    for E in envs:
        E.close()
    return rep


def shared_leg(torch, envpot, synth, n_clients=8, n_req=16, n_pts=4096):
    """One GPU shared by the processes of a node (the paper's outlook): each
    of n_clients client processes (no GPU context) evaluates its own QM/MM
    instance at n_pts host points n_req times through the server, which
    evaluates whatever requests are ready in one batched launch.  Baseline:
    the same requests one after another from one process (host points copied
    in, env_potential_eval, host values copied out).  FP32C."""
    import subprocess
    import tempfile
    import uuid
    insts = synth.batched_instances(n_clients, seed0=3100, max_points=n_pts)
    envs = [envpot.Environment.from_synth(env, precision="fp32c", neutralize=True) for env, _ in insts]
    pairs = [E.info()["n_pairs"] for E in envs]
    work = float(sum(n_req * len(p) * q for (_, p), q in zip(insts, pairs)))
    name = "bench" + uuid.uuid4().hex[:10]
    srv = envpot.Server(envs, name, n_slots=n_clients, max_points=n_pts, gather_us=20)
    with tempfile.TemporaryDirectory() as td:
        procs, answers = [], []
        for c, (_, pts) in enumerate(insts):
            req, ans = os.path.join(td, f"req{c}.npz"), os.path.join(td, f"ans{c}.npz")
            np.savez(req, env=np.array([c]), n=np.array([len(pts)]), points=pts)
            answers.append(ans)
            procs.append(subprocess.Popen([sys.executable, "-m", "paper_1011_4687_amd.server_client", name, req, ans,
                                           str(n_req)], cwd=ROOT))
        rcs = [p.wait(timeout=300) for p in procs]
        if any(rcs):
            raise RuntimeError(f"shared-GPU clients failed: {rcs}")
        res = [dict(np.load(a)) for a in answers]
    stats = srv.stats()
    srv.close()
    t_span = max(r["t_end"] for r in res) - min(r["t_start"] for r in res)
    stream = torch.cuda.current_stream()
    ref = []
    for _ in range(2):  # the first pass warms up
        ref = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(n_req):
            for E, (_, pts) in zip(envs, insts):
                v = E.eval(torch.from_numpy(pts).cuda(), stream=stream).cpu().numpy()
                if r == n_req - 1:
                    ref.append(v)
        t_serial = time.perf_counter() - t0
    diff = max(float(np.abs(r["V"] - v).max()) for r, v in zip(res, ref))
    for E in envs:
        E.close()
    rep = {
        "workload": f"{n_clients} client processes, each its own instance (atoms "
                    f"{min(e.n_nuclei for e, _ in insts)}-{max(e.n_nuclei for e, _ in insts)}), "
                    f"{n_req} requests of {n_pts} host points, FP32C",
        "shared_point_pairs_per_s": work / t_span,
        "serial_point_pairs_per_s": work / t_serial,
        "speedup_vs_serial": t_serial / t_span,
        "rounds": stats["rounds"], "requests": stats["requests"],
        "requests_per_round": stats["requests"] / max(stats["rounds"], 1),
        "max_abs_diff_vs_serial": diff,
    }
    log(f"[bench] shared GPU: {n_clients} clients, {work / t_span:.4g} pp/s vs serial {work / t_serial:.4g} "
        f"({t_serial / t_span:.2f}x), {rep['requests_per_round']:.1f} requests per launch, max diff {diff:.2e}")
    return rep


def cells_leg(args, torch, envpot, synth):
    """The paper's own form of the environment: 19 nuclei and 268,398
    point-charge cells.  Batched throughput (131,072 points per call) and the
    single-point latency of the paper's QMC loop (one electron position per
    call), for the full-device decomposition and the paper's 120 x 256 one;
    checked against the cell-sum oracle on 16 points."""
    from oracle import cells_oracle as CO
    env, pts = synth.cell_workload()
    x = torch.from_numpy(pts).cuda()
    n, m = len(pts), env.n_cells
    rep = {"workload": f"cells: {len(env.Z)} nuclei, {m} point-charge cells (h = {env.h} bohr), "
                       f"{n} points in the 3-bohr QM sphere"}
    rng = np.random.default_rng(2024)
    cidx = np.sort(rng.choice(n, size=16, replace=False))
    Vc, _, _, Ac = CO.potential(env.xyz, env.Z, env.cells, pts[cidx])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for prec in ("fp32c", "fp64"):
            E = envpot.CellEnvironment.from_synth(env, precision=prec)
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            ms, _ = time_calls(lambda st: E.eval(x, out=out, stream=st), args.steps, args.warmup, torch, side)
            r = {"point_cell_evals_per_s": n * m / (ms * 1e-3), "ms_per_step": ms}
            err = np.abs(out.cpu().numpy()[cidx] - Vc)
            r["accuracy_vs_oracle_16"] = {"max_abs_err": float(err.max()), "max_rel_to_A": float((err / Ac).max())}
            one = torch.empty(1, dtype=torch.float64, device="cuda")
            host = torch.from_numpy(np.ascontiguousarray(pts[:256]))
            for mode in (0, 1):
                for j in range(32):
                    E.eval_single(x[j], one, mode=mode)
                k = 2000
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(side)
                for j in range(k):
                    E.eval_single(x[j % n], one, mode=mode)
                e1.record(side)
                side.synchronize()
                p1 = torch.empty(3, dtype=torch.float64, device="cuda")
                t0 = time.perf_counter()
                kk = 256
                for j in range(kk):
                    p1.copy_(host[j])
                    E.eval_single(p1, one, mode=mode)
                    one.item()
                r[f"single_point_mode{mode}_us"] = e0.elapsed_time(e1) * 1e3 / k
                r[f"single_point_mode{mode}_roundtrip_us"] = (time.perf_counter() - t0) * 1e6 / kk
                # resident kernel: host position in, host V out, no launch per move
                # (the time includes the Python call into the library)
                E.resident_start(mode=mode, idle_s=10.0)
                hp = pts[:kk]
                for j in range(32):
                    E.resident_eval(hp[j])
                t0 = time.perf_counter()
                vres = [E.resident_eval(hp[j]) for j in range(kk)]
                r[f"resident_mode{mode}_roundtrip_us"] = (time.perf_counter() - t0) * 1e6 / kk
                E.resident_stop()
                same = []
                for j in range(8):
                    p1.copy_(host[j])
                    E.eval_single(p1, one, mode=mode)
                    same.append(one.item() == vres[j])
                r[f"resident_mode{mode}_equals_single"] = bool(all(same))
            rep[prec] = r
            log(f"[bench] cells {prec}: {ms:.3f} ms per {n} points; one point "
                f"{r['single_point_mode0_us']:.1f} / {r['single_point_mode1_us']:.1f} us per launch, "
                f"host round trip {r['single_point_mode0_roundtrip_us']:.1f} us, resident "
                f"{r['resident_mode0_roundtrip_us']:.1f} / {r['resident_mode1_roundtrip_us']:.1f} us; "
                f"{r['accuracy_vs_oracle_16']}")
            E.close()
    torch.cuda.synchronize()
    return rep


def surrogate1000_leg(args, torch, envpot, synth):
    """Secondary: the 1000-atom surrogate workload.  The network covers the
    6-bohr region, trained on 2M samples of the exact FP64 kernel; evaluated
    with its gate on 1,000,000 points in the region plus 65,536 points in the
    6..8-bohr shell (which the gate sends to the exact FP32C kernel), against
    the exact FP32C kernel on the same points and the stored oracle sample."""
    env, _ = synth.workload("surrogate", n_points=1)
    _, infer, outer = synth.surrogate_sets(n_train=1, n_infer=1_000_000, n_out=65536)
    pts = np.ascontiguousarray(np.concatenate([infer, outer]))
    n = len(pts)
    x = torch.from_numpy(pts).cuda()
    fb = envpot.Environment.from_synth(env, precision="fp32c", neutralize=True)
    te = envpot.Environment.from_synth(env, precision="fp64", neutralize=True)
    npairs = fb.info()["n_pairs"]
    S = envpot.Surrogate(fb, envpot.fourier_matrix(1004, 0.25), envpot.init_params(1004), radius=6.0)
    t0 = time.perf_counter()
    S.train(te, n_train=args.sur1000_train, epochs=args.sur1000_epochs, batch=8192, lr=2e-3, lr_final=1e-5,
            poly_degree=8)
    t_train = time.perf_counter() - t0
    si = S.info()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ms_exact, _ = time_calls(lambda st: fb.eval(x, out=out, stream=st), 3, 1, torch)
    V_exact = out.cpu().numpy()
    used = torch.empty(n, dtype=torch.uint8, device="cuda")
    ms, _ = time_calls(lambda st: S.eval(x, stream=st, out=out, used=used), args.steps, args.warmup, torch)
    nfb = S.info()["last_eval_fallback"]
    Vs = out.cpu().numpy()
    ms_net, _ = time_calls(lambda st: S.predict(x, stream=st, out=out), 5, 1, torch)
    saved = (ms_exact - ms) * 1e-3
    rep = {
        "workload": f"surrogate: {env.n_nuclei} atoms, {npairs} screened pairs, network radius 6 bohr; "
                    f"{len(infer)} points in the region + {len(outer)} in the 6-8 bohr shell",
        "point_pairs_per_s": n * npairs / (ms * 1e-3), "ms_per_step": ms, "network_ms": ms_net,
        "exact_fp32c_ms_per_step": ms_exact, "speedup_vs_fp32c": ms_exact / ms,
        "fallback_fraction": nfb / n, "gate_pass_volume_fraction": si["gate_pass_volume_fraction"],
        "gate_max_validation_err": si["gate_max_err_passed"], "train_total_s": t_train,
        "break_even_evaluations": t_train / saved if saved > 0 else None,
        "vs_fp32c_kernel_all_points": {"max_abs_diff": float(np.abs(Vs - V_exact).max()), "n": n},
    }
    path = os.path.join(ROOT, "tests", "golden", "surrogate_oracle_16384.npz")
    if os.path.exists(path):
        g = dict(np.load(path))
        if str(g["env_digest"]) != env.digest() or str(g["points_digest"]) != synth.digest(pts):
            raise RuntimeError("surrogate_oracle_16384.npz does not belong to this workload")
        rep["accuracy_vs_oracle_16384"] = errors(Vs[g["idx"]], g["V"], g["A"])
        rep["fp32c_accuracy_vs_oracle_16384"] = errors(V_exact[g["idx"]], g["V"], g["A"])
    log(f"[bench] surrogate (1000 atoms): {ms:.2f} ms vs exact FP32C {ms_exact:.2f} ms, fallback {nfb / n:.3f}, "
        f"train {t_train:.1f} s; {rep.get('accuracy_vs_oracle_16384')}")
    S.close()
    fb.close()
    te.close()
    return rep


def cpu_baseline(args, large):
    """The FP64 oracle (screened, as the library) timed on the host cores on
    a bounded seeded sample of the headline points: all cores, then one."""
    from oracle import oracle as O
    env, pts, info = large["env"], large["pts"], large["info"]
    rng = np.random.default_rng(12345)
    sc = O.neutral_scales(env)
    cores = min(os.cpu_count() or 1, 16)
    idx = np.sort(rng.choice(len(pts), size=args.cpu_sample, replace=False))
    t0 = time.perf_counter()
    O.potential(env, pts[idx], scale=sc, screen=True, nthreads=cores)
    t_all = time.perf_counter() - t0
    idx1 = idx[: args.cpu_sample_1core]
    t0 = time.perf_counter()
    O.potential(env, pts[idx1], scale=sc, screen=True, nthreads=1)
    t_one = time.perf_counter() - t0
    npairs = info["n_pairs"]
    rep = {"value": len(idx) * npairs / t_all, "unit": "point-pair evals/s", "cores": cores, "kind": "oracle",
           "sample": f"{len(idx)} of the {len(pts)} large-workload points (seeded), screened FP64 oracle, "
                     f"{t_all:.1f} s on {cores} threads",
           "one_core": {"value": len(idx1) * npairs / t_one, "unit": "point-pair evals/s", "cores": 1,
                        "sample": f"the first {len(idx1)} of those points, {t_one:.1f} s on 1 thread"}}
    log(f"[bench] oracle: {rep['value']:.4g} pp/s on {cores} threads, {rep['one_core']['value']:.4g} on 1")
    return rep


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sigma", type=float, default=0.25,
                    help="Fourier-feature frequency scale of the large surrogate (1/bohr)")
    ap.add_argument("--sur-epochs", type=int, default=120, help="large surrogate: training epochs over 2M samples")
    ap.add_argument("--sur-lr", type=float, default=3e-3, help="large surrogate: initial Adam learning rate")
    ap.add_argument("--sur1000-train", type=int, default=2_000_000,
                    help="1000-atom surrogate leg: training samples (profiling runs may shrink it)")
    ap.add_argument("--sur1000-epochs", type=int, default=30, help="1000-atom surrogate leg: training epochs")
    ap.add_argument("--r-near", type=float, default=15.0,
                    help="large surrogate: fragments with an atom within this radius (bohr) are evaluated "
                         "exactly and added; the network covers the rest")
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="points of the oracle's all-core CPU-baseline sample")
    ap.add_argument("--cpu-sample-1core", type=int, default=4,
                    help="points of the oracle's one-core sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip both surrogate legs")
    ap.add_argument("--large-paths", default="fp32c,fp64",
                    help="exact paths timed on the large workload (the surrogate needs both); profiling runs "
                         "may narrow this")
    ap.add_argument("--legs", default="mid,batched,cells,shared,surrogate1000",
                    help="secondary legs to run (comma list; empty for none)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(points would be sharded across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1011_4687_amd import envpot, synth
    from paper_1011_4687_amd import workcount as wc

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    large = large_leg(args, torch, envpot, synth, wc)
    paths = large["paths"]
    info = large["info"]
    n = len(large["pts"])
    legs = [s for s in args.legs.split(",") if s]
    secondary = {}
    if "mid" in legs:
        secondary["mid"] = mid_leg(args, torch, envpot, synth, wc)
    if "batched" in legs:
        secondary["batched"] = batched_leg(args, torch, envpot, synth)
    if "cells" in legs:
        secondary["cells"] = cells_leg(args, torch, envpot, synth)
    if "shared" in legs:
        secondary["shared"] = shared_leg(torch, envpot, synth)
    if "surrogate1000" in legs and not args.no_surrogate:
        secondary["surrogate1000"] = surrogate1000_leg(args, torch, envpot, synth)

    if args.copy_calibration:
        # plain copy of known size: 256 MiB read + 256 MiB written per launch
        a = torch.ones(256 << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 x 256 MiB device copies")

    if "fp32c" not in paths:
        # a narrowed run (profiling): no headline, the legs that ran
        print(json.dumps({"metric": METRIC, "value": None, "paths": paths, "secondary": secondary}), flush=True)
        return
    head = paths["fp32c"]
    flops = wc.eval_flops(n, info["n_pairs_by_L"], info["n_nuclei"])
    achieved = flops / (head["kernel_ms"] * 1e-3)
    counters = profile_record("k_potential_large_counters")
    result = {
        "metric": METRIC,
        "value": head["point_pairs_per_s"],
        "unit": "point-pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"large: {info['n_nuclei']} atoms in {large['env'].n_fragments} neutral 10-atom "
                        f"fragments, contracted s/p/d basis (nbf {large['env'].nbf}), {info['n_pairs']} "
                        f"screened primitive pairs, {n} points (65536 walkers x 16 electrons) in the 8-bohr "
                        f"QM sphere; FP32C kernel (value), FP64 kernel and surrogate with fallback in paths",
            "n_points": n,
            "n_pairs": info["n_pairs"],
            "pairs_by_L": info["n_pairs_by_L"],
            "n_nuclei": info["n_nuclei"],
            "path": "fp32c",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "traffic": counters["traffic_bytes_per_dispatch"] if counters else None,
            "kernel": "k_potential<4,false>",
            "kernel_ms": head["kernel_ms"],
            "flops_basis": "McMurchie-Davidson-equivalent flops per point-pair (recursion, Boys, contraction); "
                           "the kernel evaluates far pairs by an exact multipole polynomial and merged "
                           "same-centre clusters, which execute fewer, so this is a work rate, not issue use",
            "issue": {k: counters.get(k) for k in ("valu_issue_vs_probe", "valubusy_rocprof",
                                                     "probe_valubusy_rocprof", "probe_issue_vs_nominal",
                                                     "lds_bank_conflict_rocprof")} if counters else None,
            "issue_basis": "committed counter record of this kernel (profiles/k_potential_large_counters.json): "
                           "VALU wave-instructions per second against the v_fma_f32 probe of the same counter "
                           "pass, rocprof VALUBusy of both" if counters else None,
        },
        "paths": paths,
        "secondary": secondary,
    }
    try:
        pk = envpot.peak_probe()
        result["peak_probe"] = {"fp32_fma_tflops": pk["fp32_fma_tflops"], "fp64_fma_tflops": pk["fp64_fma_tflops"],
                                "rsq_f32_per_s": pk["rsq_f32_per_s"]}
        log(f"[bench] peak probe: FP32 FMA {pk['fp32_fma_tflops']:.1f} TFLOP/s, "
            f"FP64 FMA {pk['fp64_fma_tflops']:.1f} TFLOP/s, rsq {pk['rsq_f32_per_s']:.3g}/s")
    except envpot.EnvError as e:
        log(f"[bench] peak probe failed: {e}")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, large)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput of the environment potential on one MI355X.

A step is one evaluation of V(r) for the whole point batch of the workload
(nuclear term, Boys function, Hermite recursion and contraction, FP64
cancellation sums, output), with the pair list already on the device and the
points already in HBM.  The metric is point-pair evaluations per second:
n_points x n_pairs (unique screened primitive shell pairs) / time per step.

Default workload "mid": 200 environment atoms in 20 neutral 10-atom fragments,
contracted s/p/d shells, 375,461 screened pairs, 131,072 points
(4096 walkers x 32 electrons) in the 8-bohr QM sphere.  The headline path is
FP32C; the FP64 path is timed beside it.  The CPU-baseline leg times the FP64
oracle on a bounded sample of the same points and reports the GPU paths'
errors on that sample.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "point-pair evals/s at ≤1e-5 Ha max err: FP64 vs FP32 vs MLP surrogate, 1 GPU"

PEAK_FP32 = 157.3e12   # MI355X FP32 vector (published, packed)
PEAK_FP64 = 78.6e12    # MI355X FP64 vector


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per dispatch of the FP32C kernel from the committed counter
    runs, or None when the kernel sources changed since they were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "k_potential_mid_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for s in rec["kernel_sources"]:
            h.update(open(os.path.join(root, s), "rb").read())
        if h.hexdigest() != rec["kernel_source_sha256"]:
            return None
        return rec["traffic_bytes_per_dispatch"]
    except (OSError, KeyError, ValueError):
        return None


def time_path(E, x, out, steps, warmup, torch):
    for _ in range(warmup):
        E.eval(x, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in evs:
        s.record(stream)
        E.eval(x, out=out, stream=stream)
        e.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ms = [s.elapsed_time(e) for s, e in evs]
    return wall, float(np.mean(ms))


def time_field(E, x, out, steps, warmup, torch):
    """Mean device time (ms) of one field evaluation, HIP events on a side
    stream around each call."""
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            E.eval_field(x, out=out, stream=stream)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for s, e in evs:
            s.record(stream)
            E.eval_field(x, out=out, stream=stream)
            e.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([s.elapsed_time(e) for s, e in evs]))


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
    root = os.path.dirname(os.path.abspath(__file__))
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
                                           str(n_req)], cwd=root))
        rcs = [p.wait(timeout=300) for p in procs]
        if any(rcs):
            raise RuntimeError(f"shared-GPU clients failed: {rcs}")
        res = [dict(np.load(a)) for a in answers]
    stats = srv.stats()
    srv.close()
    t_span = max(r["t_end"] for r in res) - min(r["t_start"] for r in res)
    # baseline: the same requests serially from this process
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


def cells_leg(torch, envpot, synth, steps, warmup):
    """The paper's own form of the environment: 19 nuclei and 268,398
    point-charge cells.  Batched throughput (131,072 points per call) and the
    single-point latency of the paper's QMC loop (one electron position per
    call), for the full-device decomposition and the paper's 120 x 256 one."""
    env, pts = synth.cell_workload()
    x = torch.from_numpy(pts).cuda()
    n, m = len(pts), env.n_cells
    rep = {"workload": f"cells: {len(env.Z)} nuclei, {m} point-charge cells (h = {env.h} bohr), "
                       f"{n} points in the 3-bohr QM sphere"}
    values = {}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for prec in ("fp32c", "fp64"):
            E = envpot.CellEnvironment.from_synth(env, precision=prec)
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            wall, ms = time_path(E, x, out, steps, warmup, torch)
            r = {"point_cell_evals_per_s": n * m / (ms * 1e-3), "ms_per_step": ms}
            values[prec] = out.cpu().numpy()
            # single point: back-to-back launches on the device, then the
            # host round trip of the paper's loop (position in, value out)
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
                dev_us = e0.elapsed_time(e1) * 1e3 / k
                p1 = torch.empty(3, dtype=torch.float64, device="cuda")
                t0 = time.perf_counter()
                kk = 256
                for j in range(kk):
                    p1.copy_(host[j])
                    E.eval_single(p1, one, mode=mode)
                    one.item()
                rt_us = (time.perf_counter() - t0) * 1e6 / kk
                r[f"single_point_mode{mode}_us"] = dev_us
                r[f"single_point_mode{mode}_roundtrip_us"] = rt_us
            rep[prec] = r
            log(f"[bench] cells {prec}: {ms:.3f} ms per {n} points ({r['point_cell_evals_per_s']:.4g} "
                f"point-cell/s); one point: {r['single_point_mode0_us']:.1f} us (full device), "
                f"{r['single_point_mode1_us']:.1f} us (120 x 256), round trip "
                f"{r['single_point_mode0_roundtrip_us']:.1f} / {r['single_point_mode1_roundtrip_us']:.1f} us")
            E.close()
    torch.cuda.synchronize()
    return {"report": rep, "env": env, "points": pts, "values": values}


def surrogate_leg(torch, envpot, synth):
    """Learned surrogate on its own workload: 1000 atoms (box 68.4 bohr), the
    network covering the 6-bohr region, trained on 2M samples of the exact FP64
    kernel; evaluated with its gate on 1,000,000 points in the region plus
    65,536 points in the 6..8-bohr shell (which the gate sends to the exact
    FP32C kernel), against the exact FP32C kernel on the same points."""
    env, _ = synth.workload("surrogate", n_points=1)
    _, infer, outer = synth.surrogate_sets(n_train=1, n_infer=1_000_000, n_out=65536)
    pts = np.ascontiguousarray(np.concatenate([infer, outer]))
    x = torch.from_numpy(pts).cuda()
    fb = envpot.Environment.from_synth(env, precision="fp32c", neutralize=True)
    te = envpot.Environment.from_synth(env, precision="fp64", neutralize=True)
    npairs = fb.info()["n_pairs"]
    S = envpot.Surrogate(fb, envpot.fourier_matrix(1004, 0.25), envpot.init_params(1004), radius=6.0)
    t0 = time.perf_counter()
    S.train(te, n_train=2_000_000, epochs=30, batch=8192, lr=2e-3, lr_final=1e-5, poly_degree=8)
    t_train = time.perf_counter() - t0
    info = S.info()
    out = torch.empty(len(pts), dtype=torch.float64, device="cuda")
    _, ms_exact = time_path(fb, x, out, 3, 1, torch)
    V_exact = out.cpu().numpy()
    S.eval(x)
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_ev.record()
        V, used = S.eval(x)
        e_ev.record()
        torch.cuda.synchronize()
        times.append(s_ev.elapsed_time(e_ev))
    ms_sur = float(np.mean(times))
    used = used.cpu().numpy().astype(bool)
    n = len(pts)
    saved_per_eval = (ms_exact - ms_sur) * 1e-3
    report = {
        "workload": f"surrogate: {env.n_nuclei} atoms, {npairs} screened pairs, network radius "
                    f"6 bohr; {len(infer)} points in the region + {len(outer)} in the 6-8 bohr shell",
        "n_points": n,
        "point_pairs_per_s": n * npairs / (ms_sur * 1e-3),
        "ms_per_step": ms_sur,
        "exact_fp32c_ms_per_step": ms_exact,
        "exact_fp32c_point_pairs_per_s": n * npairs / (ms_exact * 1e-3),
        "speedup_vs_fp32c": ms_exact / ms_sur,
        "fallback_fraction": float(used.mean()),
        "gate_pass_volume_fraction": info["gate_pass_volume_fraction"],
        "gate_max_validation_err": info["gate_max_err_passed"],
        "baseline_rms": info["baseline_rms"],
        "teacher_s": info["teacher_seconds"],
        "train_s": info["train_seconds"],
        "gate_s": info["gate_seconds"],
        "train_total_s": t_train,
        "break_even_evaluations": (t_train / saved_per_eval) if saved_per_eval > 0 else None,
    }
    log(f"[bench] surrogate: {ms_sur:.2f} ms vs exact FP32C {ms_exact:.2f} ms, "
        f"fallback {used.mean():.3f}, train {t_train:.1f}s")
    V_sur = V.cpu().numpy()
    S.close()
    fb.close()
    te.close()
    return {"report": report, "env": env, "points": pts, "V_surrogate": V_sur, "V_exact": V_exact}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--cpu-sample", type=int, default=96,
                    help="points of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paths", default="fp32c,fp64")
    ap.add_argument("--no-cells", action="store_true",
                    help="skip the cell-sum leg (the paper's own form of the environment)")
    ap.add_argument("--no-field", action="store_true",
                    help="skip the field leg (E = -grad V with V on the same workload)")
    ap.add_argument("--no-shared", action="store_true",
                    help="skip the shared-GPU leg (client processes feeding one server)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-surrogate leg (1000-atom surrogate workload)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(points would be sharded across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1011_4687_amd import envpot, synth
    from paper_1011_4687_amd.workcount import eval_field_flops, eval_flops

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    env, pts = synth.workload(args.workload)
    n = pts.shape[0]
    x = torch.from_numpy(pts).cuda()
    log(f"[bench] workload {args.workload}: {env.n_nuclei} atoms, nbf {env.nbf}, {n} points")

    paths = {}
    outs = {}
    fields = {}
    info = None
    for prec in args.paths.split(","):
        t0 = time.perf_counter()
        E = envpot.Environment.from_synth(env, precision=prec, neutralize=True)
        t_create = time.perf_counter() - t0
        info = E.info()
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        wall, ms = time_path(E, x, out, args.steps, args.warmup, torch)
        npairs = info["n_pairs"]
        flops = eval_flops(n, info["n_pairs_by_L"], info["n_nuclei"])
        paths[prec] = {
            "point_pairs_per_s": n * npairs / (ms * 1e-3),
            "ms_per_step": ms,
            "wall_ms_per_step": wall * 1e3,
            "create_s": t_create,
            "tflops_algorithmic": flops / (ms * 1e-3) / 1e12,
        }
        outs[prec] = out.cpu().numpy()
        log(f"[bench] {prec}: {ms:.3f} ms/step, {paths[prec]['point_pairs_per_s']:.4g} pp/s")
        if not args.no_field:
            # the field E = -grad V (with V) of the same handle at the same points
            fout = torch.empty((n, 4), dtype=torch.float64, device="cuda")
            fms = time_field(E, x, fout, args.steps, args.warmup, torch)
            fflops = eval_field_flops(n, info["n_pairs_by_L"], info["n_nuclei"])
            paths[prec]["field"] = {
                "point_pairs_per_s": n * npairs / (fms * 1e-3),
                "ms_per_step": fms,
                "tflops_algorithmic": fflops / (fms * 1e-3) / 1e12,
            }
            fields[prec] = fout.cpu().numpy()
            log(f"[bench] {prec} field: {fms:.3f} ms/step, {n * npairs / (fms * 1e-3):.4g} pp/s, "
                f"{fflops / (fms * 1e-3) / 1e12:.1f} TFLOP/s algorithmic")
        # a new density with the same blocks (each fragment block rescaled),
        # refolded on the device, against building the handle again
        rowp, col, val = env.density_csr(None)
        P2 = (rowp, col, val * 1.05)
        t_upd = []
        for _ in range(3):
            t0 = time.perf_counter()
            E.update_density(P2)
            t_upd.append(time.perf_counter() - t0)
        paths[prec]["density_update_ms"] = float(np.median(t_upd)) * 1e3
        log(f"[bench] {prec} density update: {paths[prec]['density_update_ms']:.1f} ms "
            f"(create {t_create * 1e3:.0f} ms)")
        E.close()

    cells = None
    if not args.no_cells:
        cells = cells_leg(torch, envpot, synth, args.steps, args.warmup)
        paths["cells"] = cells["report"]

    if not args.no_shared:
        paths["shared"] = shared_leg(torch, envpot, synth)

    sur = None
    if not args.no_surrogate and "fp32c" in args.paths.split(","):
        sur = surrogate_leg(torch, envpot, synth)
        paths["surrogate"] = sur["report"]

    if args.copy_calibration:
        # plain copy of known size: 256 MiB read + 256 MiB written per launch
        a = torch.ones(256 << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 x 256 MiB device copies")

    head = "fp32c" if "fp32c" in paths else list(paths)[0]
    flops = eval_flops(n, info["n_pairs_by_L"], info["n_nuclei"])
    ms = paths[head]["ms_per_step"]
    peak = PEAK_FP32 if head == "fp32c" else PEAK_FP64
    achieved = flops / (ms * 1e-3)
    result = {
        "metric": METRIC,
        "value": paths[head]["point_pairs_per_s"],
        "unit": "point-pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if head == "fp32c" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {env.n_nuclei} atoms in {env.n_fragments} neutral "
                        f"fragments, contracted s/p/d basis (nbf {env.nbf}), "
                        f"{info['n_pairs']} screened primitive pairs, {n} points in the "
                        f"{8.0 if args.workload != 'tiny' else 4.0}-bohr QM sphere",
            "n_points": n,
            "n_pairs": info["n_pairs"],
            "pairs_by_L": info["n_pairs_by_L"],
            "n_nuclei": info["n_nuclei"],
            "path": head,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": peak / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": measured_traffic() if (head == "fp32c" and args.workload == "mid") else None,
        },
        "paths": paths,
    }

    # on-device peak probes: what independent FMA / rsq streams sustain here
    try:
        pk = envpot.peak_probe()
        result["peak_probe"] = {
            "fp32_fma_tflops": pk["fp32_fma_tflops"],
            "fp64_fma_tflops": pk["fp64_fma_tflops"],
            "rsq_f32_per_s": pk["rsq_f32_per_s"],
            "fp32c_achieved_frac": (flops / (paths["fp32c"]["ms_per_step"] * 1e-3) / 1e12)
            / pk["fp32_fma_tflops"] if "fp32c" in paths else None,
            "fp64_achieved_frac": (flops / (paths["fp64"]["ms_per_step"] * 1e-3) / 1e12)
            / pk["fp64_fma_tflops"] if "fp64" in paths else None,
        }
        log(f"[bench] peak probe: FP32 FMA {pk['fp32_fma_tflops']:.1f} TFLOP/s, "
            f"FP64 FMA {pk['fp64_fma_tflops']:.1f} TFLOP/s, rsq {pk['rsq_f32_per_s']:.3g}/s")
    except envpot.EnvError as e:
        log(f"[bench] peak probe failed: {e}")

    if not args.no_cpu_baseline:
        # CPU-baseline leg: the FP64 oracle on a bounded sample of the same points
        from oracle import oracle as O
        rng = np.random.default_rng(12345)
        idx = np.sort(rng.choice(n, size=min(args.cpu_sample, n), replace=False))
        sc = O.neutral_scales(env)
        cores = os.cpu_count() or 1
        t0 = time.perf_counter()
        Vo, Vn, Ve, A = O.potential(env, pts[idx], scale=sc, screen=True, nthreads=cores)
        t_or = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": len(idx) * info["n_pairs"] / t_or,
            "unit": "point-pair evals/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"{len(idx)} of the {n} points (seeded), screened FP64 oracle, "
                      f"{t_or:.1f} s on {cores} threads",
        }
        acc = {}
        for prec, V in outs.items():
            err = np.abs(V[idx] - Vo)
            acc[prec] = {"max_abs_err": float(err.max()), "rms_err": float(np.sqrt(np.mean(err ** 2))),
                         "max_rel_to_A": float((err / A).max())}
        if sur is not None:
            # the same oracle on a sample of the surrogate workload's points
            k = min(48, len(sur["points"]))
            sidx = np.sort(rng.choice(len(sur["points"]), size=k, replace=False))
            sc2 = O.neutral_scales(sur["env"])
            Vo2, _, _, _ = O.potential(sur["env"], sur["points"][sidx], scale=sc2, screen=False,
                                       nthreads=cores)
            for name, V in (("surrogate", sur["V_surrogate"]), ("surrogate_workload_fp32c", sur["V_exact"])):
                err = np.abs(V[sidx] - Vo2)
                acc[name] = {"max_abs_err": float(err.max()),
                             "rms_err": float(np.sqrt(np.mean(err ** 2))), "n_checked": int(k)}
        if fields:
            # the field oracle on a smaller sample of the same points
            fidx = idx[: max(8, len(idx) // 4)]
            t0 = time.perf_counter()
            Eo, AE = O.field(env, pts[fidx], scale=sc, screen=True, nthreads=cores)
            t_f = time.perf_counter() - t0
            result["cpu_baseline"]["field"] = {
                "value": len(fidx) * info["n_pairs"] / t_f, "unit": "point-pair field evals/s",
                "cores": cores, "sample": f"{len(fidx)} of the {n} points, screened FP64 field oracle, "
                                          f"{t_f:.1f} s on {cores} threads"}
            for prec, F in fields.items():
                err = np.abs(F[fidx, 1:] - Eo).max(axis=1)
                acc[f"field_{prec}"] = {"max_abs_err": float(err.max()),
                                        "max_rel_to_AE": float((err / AE).max()), "n_checked": len(fidx)}
        if cells is not None:
            # the cell-sum oracle, one host core, on a sample of that workload
            from oracle import cells_oracle as CO
            cenv, cpts = cells["env"], cells["points"]
            cidx = np.sort(rng.choice(len(cpts), size=16, replace=False))
            t0 = time.perf_counter()
            Vc, _, _, Ac = CO.potential(cenv.xyz, cenv.Z, cenv.cells, cpts[cidx])
            t_c = time.perf_counter() - t0
            result["cpu_baseline"]["cells"] = {
                "value": len(cidx) * cenv.n_cells / t_c, "unit": "point-cell evals/s", "cores": 1,
                "ms_per_point": t_c * 1e3 / len(cidx),
                "sample": f"{len(cidx)} of the {len(cpts)} cell-workload points, FP64 cell-sum oracle (numpy)"}
            for prec, V in cells["values"].items():
                err = np.abs(V[cidx] - Vc)
                acc[f"cells_{prec}"] = {"max_abs_err": float(err.max()),
                                        "max_rel_to_A": float((err / Ac).max()), "n_checked": len(cidx)}
        result["accuracy_vs_oracle"] = acc
        log(f"[bench] oracle {t_or:.1f}s; accuracy {acc}")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

"""Segment far-field boxes: an evaluation that skips the per-pair near test
for every segment whose box all points of a wave are beyond agrees with one
that tests every pair (ENVPOT_NO_FARBOX=1 at create): FP64 bit for bit;
FP32C, which also forms the coordinate differences of such segments from a
wave origin (at most 3 FP32 ulps of |X| instead of 1), within 2e-6 Ha.  On
the mid and 5000-atom workloads, batched, without allocation, and with
points far outside the molecule (every segment all far) and inside it (few
segments all far)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

_cache = {}


def _workload(name, n_points):
    if name not in _cache:
        from paper_1011_4687_amd import synth
        _cache[name] = synth.workload(name, n_points=n_points)
    return _cache[name]


def _pair(env, **kw):
    from paper_1011_4687_amd.envpot import Environment
    A = Environment.from_synth(env, **kw)
    os.environ["ENVPOT_NO_FARBOX"] = "1"
    try:
        B = Environment.from_synth(env, **kw)
    finally:
        os.environ.pop("ENVPOT_NO_FARBOX")
    return A, B


def _eval(E, pts):
    import torch
    v = E.eval(torch.from_numpy(np.ascontiguousarray(pts)).cuda())
    torch.cuda.synchronize()
    return v.cpu().numpy()


TOL32 = 2e-6  # Ha: FP32C origin form against the rounded exact difference


def _agree(va, vb, precision, what=""):
    if precision == "fp64":
        bad = np.flatnonzero(va != vb)
        assert bad.size == 0, f"{what}: {bad.size} of {va.size} potentials differ, first at {bad[:8]}"
    else:
        d = np.abs(va - vb)
        print(f"[farbox] {what} fp32c max |diff| {d.max():.3e} Ha, rms {np.sqrt(np.mean(d * d)):.3e}", flush=True)
        assert d.max() <= TOL32


def _check(A, B, pts, precision, what=""):
    _agree(_eval(A, pts), _eval(B, pts), precision, what)


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
@pytest.mark.parametrize("where", ["workload", "far_outside", "mixed"])
def test_mid_boxes_agree(precision, where):
    print(f"[farbox] mid {precision} {where}", flush=True)
    env, pts = _workload("mid", 8192)
    if where == "far_outside":
        pts = pts + np.array([40.0, -25.0, 30.0])
    elif where == "mixed":
        rng = np.random.default_rng(3)
        lo, hi = env.xyz.min(0) - 4.0, env.xyz.max(0) + 4.0
        pts = np.concatenate([pts[:4000], rng.uniform(lo, hi, (3000, 3)), pts[4000:5001] + 15.0])
    A, B = _pair(env, precision=precision, neutralize=True)
    try:
        _check(A, B, pts, precision, f"mid {where}")
    finally:
        A.close()
        B.close()


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_large_boxes_agree(precision):
    print(f"[farbox] large {precision}", flush=True)
    env, pts = _workload("large", 65536)
    A, B = _pair(env, precision=precision, neutralize=True)
    try:
        _check(A, B, pts, precision, "large")
    finally:
        A.close()
        B.close()


def test_batched_and_noalloc_boxes_agree():
    import torch
    from paper_1011_4687_amd.envpot import Batch
    print("[farbox] batched and noalloc", flush=True)
    env, pts = _workload("mid", 8192)
    env2, _ = _workload("tiny", 1024)
    A, B = _pair(env, precision="fp32c", neutralize=True)
    A2, B2 = _pair(env2, precision="fp32c")
    ba, bb = Batch([A, A2]), Batch([B, B2])
    try:
        x = [torch.from_numpy(pts).cuda(), torch.from_numpy(pts[:5000] + 2.0).cuda()]
        oa, ob = ba.eval(x), bb.eval(x)
        torch.cuda.synchronize()
        for u, v in zip(oa, ob):
            _agree(u.cpu().numpy(), v.cpu().numpy(), "fp32c", "batched")
        n = 3000
        xa = torch.from_numpy(pts[:n]).cuda()
        ua = torch.empty(n, dtype=torch.float64, device="cuda")
        ub = torch.empty_like(ua)
        A.eval_noalloc(xa, ua)
        B.eval_noalloc(xa, ub)
        torch.cuda.synchronize()
        _agree(ua.cpu().numpy(), ub.cpu().numpy(), "fp32c", "noalloc")
    finally:
        ba.close()
        bb.close()
        for E in (A, B, A2, B2):
            E.close()


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_field_boxes_agree(precision):
    """The field kernel with segment boxes against every pair tested: bit for
    bit in both precisions (the field keeps the exact coordinate difference
    in all-far segments)."""
    import torch
    print(f"[farbox] field mid {precision}", flush=True)
    env, pts = _workload("mid", 8192)
    A, B = _pair(env, precision=precision, neutralize=True)
    try:
        x = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
        fa = A.eval_field(x).cpu().numpy()
        fb = B.eval_field(x).cpu().numpy()
        bad = np.flatnonzero((fa != fb).any(axis=1))
        assert bad.size == 0, f"{bad.size} of {len(pts)} field rows differ, first at {bad[:8]}"
    finally:
        A.close()
        B.close()

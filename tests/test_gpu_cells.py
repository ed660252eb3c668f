"""GPU parity of the cell-sum environment (the paper's own form of the field,
nuclei plus point-charge cells) through the C ABI, against the FP64 cell
oracle: FP64 within 1e-12 A(r), FP32C within 1e-5 hartree."""
import numpy as np
import pytest

from common import sample_indices

pytestmark = pytest.mark.gpu

_cache = {}


def _paper_workload():
    if "paper" not in _cache:
        from paper_1011_4687_amd import synth
        _cache["paper"] = synth.cell_workload()
    return _cache["paper"]


def _small_workload(seed=11, n_cells=3000, n_points=1000):
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-6, 6, (7, 3))
    xyz[np.linalg.norm(xyz, axis=1) < 3.5] *= 2.0
    Z = rng.choice([1.0, 6.0, 7.0, 8.0], 7)
    c = xyz[rng.integers(0, 7, n_cells)] + rng.normal(0, 0.7, (n_cells, 3))
    q = rng.uniform(0.0, 1.0, n_cells)
    cells = np.concatenate([c, (q * Z.sum() / q.sum())[:, None]], axis=1)
    u = rng.normal(size=(n_points, 3))
    pts = u / np.linalg.norm(u, axis=1)[:, None] * rng.uniform(0, 1.5, (n_points, 1))
    return xyz, Z, cells, pts


def _check(precision, V, Vo, A):
    if precision == "fp64":
        assert np.all(np.abs(V - Vo) <= 1e-12 * A), (np.abs(V - Vo) / A).max()
    else:
        assert np.abs(V - Vo).max() <= 1e-5, np.abs(V - Vo).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("n", [1, 255, 1000])
def test_small_all_points(precision, n):
    import torch
    from oracle import cells_oracle as C
    from paper_1011_4687_amd.envpot import CellEnvironment
    print(f"[cells] small {precision} n={n}", flush=True)
    xyz, Z, cells, pts = _small_workload(n_points=n)
    E = CellEnvironment(xyz, Z, cells, precision=precision)
    V = E.eval(torch.from_numpy(pts).cuda()).cpu().numpy()
    Vo, _, _, A = C.potential(xyz, Z, cells, pts)
    _check(precision, V, Vo, A)
    E.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_paper_size_batched(precision):
    """268,398 cells and 19 nuclei (the paper's benchmark shape), 131,072
    points in one call; 64 sampled points against the oracle; bitwise
    reproducible."""
    import torch
    from oracle import cells_oracle as C
    from paper_1011_4687_amd.envpot import CellEnvironment
    print(f"[cells] paper size {precision}", flush=True)
    env, pts = _paper_workload()
    E = CellEnvironment.from_synth(env, precision=precision)
    x = torch.from_numpy(pts).cuda()
    V = E.eval(x).cpu().numpy()
    V2 = E.eval(x).cpu().numpy()
    assert np.array_equal(V, V2)
    idx = sample_indices(len(pts), 64)
    Vo, _, _, A = C.potential(env.xyz, env.Z, env.cells, pts[idx])
    _check(precision, V[idx], Vo, A)
    E.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_single_point_modes(precision):
    """One electron position per launch: the full-device decomposition and
    the paper's 120 x 256 one agree with the oracle and with each other,
    repeated calls are bitwise equal (the finishing counter resets)."""
    import torch
    from oracle import cells_oracle as C
    from paper_1011_4687_amd.envpot import CellEnvironment
    print(f"[cells] single point {precision}", flush=True)
    env, pts = _paper_workload()
    E = CellEnvironment.from_synth(env, precision=precision)
    idx = sample_indices(len(pts), 16, seed=5)
    x = torch.from_numpy(np.ascontiguousarray(pts[idx])).cuda()
    out = torch.empty((2, len(idx)), dtype=torch.float64, device="cuda")
    for mode in (0, 1):
        for j in range(len(idx)):
            E.eval_single(x[j], out[mode, j:j + 1], mode=mode)
    again = torch.empty(len(idx), dtype=torch.float64, device="cuda")
    for j in range(len(idx)):
        E.eval_single(x[j], again[j:j + 1], mode=0)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.array_equal(o[0], again.cpu().numpy())
    Vo, _, _, A = C.potential(env.xyz, env.Z, env.cells, pts[idx])
    for mode in (0, 1):
        _check(precision, o[mode], Vo, A)
    batched = E.eval(x).cpu().numpy()
    tol = 1e-12 * A if precision == "fp64" else 2e-6
    assert np.all(np.abs(o[0] - batched) <= tol) and np.all(np.abs(o[1] - batched) <= tol)
    E.close()


def test_create_errors():
    from paper_1011_4687_amd.envpot import CellEnvironment, EnvError
    xyz, Z, cells, _ = _small_workload(n_cells=10, n_points=1)
    bad = cells.copy()
    bad[3, 1] = np.nan
    with pytest.raises(EnvError):
        CellEnvironment(xyz, Z, bad)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_resident_single_point(precision):
    """The resident kernel answers positions posted through host memory with
    the values of the one-launch-per-position mode, bit for bit, in both
    decompositions; it is launched again after leaving for lack of
    positions; eval before start is refused; destroy ends it."""
    import time
    import torch
    from paper_1011_4687_amd.envpot import ENV_E_STATE, CellEnvironment, EnvError
    print(f"[cells] resident single point {precision}", flush=True)
    env, pts = _paper_workload()
    E = CellEnvironment.from_synth(env, precision=precision)
    idx = sample_indices(len(pts), 16, seed=7)
    x = torch.from_numpy(np.ascontiguousarray(pts[idx])).cuda()
    with pytest.raises(EnvError) as ei:
        E.resident_eval(pts[idx[0]])
    assert ei.value.status == ENV_E_STATE
    for mode in (0, 1):
        ref = torch.empty(len(idx), dtype=torch.float64, device="cuda")
        for j in range(len(idx)):
            E.eval_single(x[j], ref[j:j + 1], mode=mode)
        torch.cuda.synchronize()
        ref = ref.cpu().numpy()
        E.resident_start(mode=mode, idle_s=5.0)
        got = np.array([E.resident_eval(pts[i]) for i in idx])
        assert np.array_equal(got, ref), (mode, np.abs(got - ref).max())
        t0 = time.perf_counter()
        for j in range(200):
            E.resident_eval(pts[idx[j % len(idx)]])
        print(f"[cells] resident mode {mode}: {(time.perf_counter() - t0) / 200 * 1e6:.1f} us per move", flush=True)
        E.resident_stop()
        if mode == 0:
            # leaves after 0.2 s without a position; the next move launches it again
            E.resident_start(mode=0, idle_s=0.2)
            assert E.resident_eval(pts[idx[0]]) == ref[0]
            time.sleep(0.6)
            assert E.resident_eval(pts[idx[1]]) == ref[1]
            E.resident_stop()
    E.resident_start(mode=1, idle_s=5.0)
    E.close()  # stops the kernel

"""Shared helpers of the test suite (inputs only; no method arithmetic)."""
import numpy as np

from paper_1011_4687_amd import synth


def sample_indices(n, k, seed=7):
    """k sorted point indices in [0, n) incl. the first and the last."""
    if k >= n:
        return np.arange(n)
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(n, size=k - 2, replace=False).tolist()) | {0, n - 1}
    return np.array(sorted(idx))


_cache = {}


def workload_scaled(name, n_points=None):
    """(env, points, P_csr) with every fragment block neutralised by the
    oracle's overlap (tests pass this explicit P to both sides)."""
    key = (name, n_points)
    if key not in _cache:
        from oracle import oracle as O
        env, pts = synth.workload(name, n_points=n_points)
        sc = O.neutral_scales(env)
        _cache[key] = (env, pts, env.density_csr(sc), sc)
    return _cache[key]

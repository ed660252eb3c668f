"""Writes the stored FP64 oracle values of the mid, batched and surrogate
workloads at the sample sizes their accuracy is stated on:

* mid (200 atoms, 131,072 points): 16,384 seeded-random points;
* batched (64 instances of 50-2000 atoms): 256 seeded-random points of
  every instance (all of them where an instance has fewer);
* surrogate (1000 atoms; 1,000,000 points in the 6-bohr region plus 65,536
  in the 6-8 bohr shell, in that order): 16,384 seeded-random points.

Each value is the screened oracle (drop rule at 1e-12, neutral fragments):
V = sum_A Z_A/|r - R_A| - sum P [mu nu|r] (the paper's Sec. II.B potential with
the density given by a density matrix), with V_nuc, V_ele and the conditioning
scale A = V_nuc + sum |terms|.  The screening change itself is checked by the
tests on a few points against the unscreened oracle.

Calls only the oracle and the input generator.  Each workload takes from
half an hour (mid) to a few hours (surrogate) of CPU time on 8 host cores.
usage: python tests/golden/make_goldens.py {mid|batched|surrogate} [threads]"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1011_4687_amd import synth  # noqa: E402

N_MID = 16384
N_SUR = 16384
N_INST = 256
CHUNK = 256


def sample(n, k, seed):
    """k distinct sorted indices of range(n) (all of them when n <= k)."""
    if n <= k:
        return np.arange(n)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=k, replace=False))


def surrogate_points():
    """The surrogate workload's evaluation points: 1,000,000 in the region
    followed by 65,536 in the 6-8 bohr shell."""
    _, infer, outer = synth.surrogate_sets(n_train=1, n_infer=1_000_000, n_out=65536)
    return np.ascontiguousarray(np.concatenate([infer, outer]))


def run_oracle(env, pts, threads, tag):
    sc = O.neutral_scales(env)
    t0 = time.time()
    out = {"V": [], "V_nuc": [], "V_ele": [], "A": []}
    for k in range(0, len(pts), CHUNK):
        v, vn, ve, a = O.potential(env, pts[k:k + CHUNK], scale=sc, screen=True, nthreads=threads)
        for key, arr in zip(("V", "V_nuc", "V_ele", "A"), (v, vn, ve, a)):
            out[key].append(arr)
        print(f"[{tag}] {min(k + CHUNK, len(pts))}/{len(pts)} points, {time.time() - t0:.0f} s", flush=True)
    res = {key: np.concatenate(v) for key, v in out.items()}
    res["scale"] = sc
    return res


def main():
    which = sys.argv[1]
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    if which == "mid":
        env, pts = synth.workload("mid")
        idx = sample(len(pts), N_MID, 16384)
        r = run_oracle(env, pts[idx], threads, "mid")
        np.savez(os.path.join(HERE, "mid_oracle_16384.npz"), idx=idx, env_digest=np.array(env.digest()),
                 points_digest=np.array(synth.digest(pts)), **r)
    elif which == "surrogate":
        env, _ = synth.workload("surrogate", n_points=1)
        pts = surrogate_points()
        idx = sample(len(pts), N_SUR, 16385)
        r = run_oracle(env, pts[idx], threads, "surrogate")
        np.savez(os.path.join(HERE, "surrogate_oracle_16384.npz"), idx=idx, env_digest=np.array(env.digest()),
                 points_digest=np.array(synth.digest(pts)), **r)
    elif which == "batched":
        insts = synth.batched_instances(64)
        rec = {}
        for i, (env, pts) in enumerate(insts):
            idx = sample(len(pts), N_INST, 3000 + i)
            r = run_oracle(env, pts[idx], threads, f"batched {i}")
            rec[f"idx{i}"] = idx
            rec[f"env_digest{i}"] = np.array(env.digest())
            rec[f"points_digest{i}"] = np.array(synth.digest(pts))
            for key in ("V", "V_nuc", "V_ele", "A", "scale"):
                rec[f"{key}{i}"] = r[key]
        np.savez(os.path.join(HERE, "batched_oracle_256.npz"), n_inst=np.array(len(insts)), **rec)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main()

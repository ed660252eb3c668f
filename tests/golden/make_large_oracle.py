"""Writes large_oracle_4096.npz: the FP64 oracle (screened at 1e-12, the
definition V = sum_A Z_A/|r - R_A| - sum P [mu nu|r] of the paper's Sec. II.B
with the density given by a density matrix) at 4096 seeded-random points of
the large workload (5000 atoms in 500 neutral fragments, 1,048,576 points).
The large workload's accuracy is stated on a 4096-point subsample; this
oracle run takes about an hour of CPU time, so its result is stored.

Calls only the oracle and the input generator.
usage: python tests/golden/make_large_oracle.py [threads]"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1011_4687_amd import synth  # noqa: E402

SEED = 4096
N_SAMPLE = 4096


def sample(n):
    rng = np.random.default_rng(SEED)
    return np.sort(rng.choice(n, size=N_SAMPLE, replace=False))


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    env, pts = synth.workload("large")
    idx = sample(len(pts))
    sc = O.neutral_scales(env)
    t0 = time.time()
    V, Vn, Ve, A = [], [], [], []
    for k in range(0, N_SAMPLE, 256):
        v, vn, ve, a = O.potential(env, pts[idx[k:k + 256]], scale=sc, screen=True, nthreads=threads)
        V.append(v)
        Vn.append(vn)
        Ve.append(ve)
        A.append(a)
        print(f"{k + 256}/{N_SAMPLE} points, {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "large_oracle_4096.npz"), idx=idx, V=np.concatenate(V), V_nuc=np.concatenate(Vn),
             V_ele=np.concatenate(Ve), A=np.concatenate(A), scale=sc,
             env_digest=np.array(env.digest()), points_digest=np.array(synth.digest(pts)))


if __name__ == "__main__":
    main()

"""A client process of a shared-GPU server (no GPU context, no torch):
attach to the server by name, send the requests listed in a .npz file
(arrays env, n, points), write the answers and the wall-clock start and end
of the request loop to another .npz file.

usage: python -m paper_1011_4687_amd.server_client NAME REQUESTS.npz ANSWERS.npz [REPEAT]"""
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np  # noqa: E402

from paper_1011_4687_amd.envpot import Client  # noqa: E402


def main():
    name, req, ans = sys.argv[1], sys.argv[2], sys.argv[3]
    repeat = int(sys.argv[4]) if len(sys.argv) > 4 else 1
    d = np.load(req)
    envs, counts, pts = d["env"], d["n"], d["points"]
    c = Client(name)
    offs = np.concatenate([[0], np.cumsum(counts)])
    outs = []
    t_start = time.time()
    t0 = time.perf_counter()
    for r in range(repeat):
        for k in range(len(envs)):
            v = c.eval(int(envs[k]), pts[offs[k]:offs[k + 1]])
            if r == repeat - 1:
                outs.append(v)
    wall = time.perf_counter() - t0
    t_end = time.time()
    c.close()
    np.savez(ans, V=np.concatenate(outs) if outs else np.zeros(0), wall=wall, t_start=t_start, t_end=t_end)


if __name__ == "__main__":
    main()

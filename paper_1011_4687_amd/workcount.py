"""Algorithmic work of the potential, for throughput and roofline figures.

The unit of work is one point x one screened primitive shell pair.  Flops
are those of the method's own steps (an FMA counts 2), independent of how the
kernels schedule them:

* distance and argument: X, Y, Z = P - C (3), R^2 (5), T = p R^2 (1): 9
* Boys values G_0..G_L: 3L + 4 besides the one transcendental
* Hermite recursion R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{tuv}:
  1 flop when t = 0, 2 when t = 1 (one FMA), 3 when t >= 2, summed over
  every intermediate of the recursion for total angular momentum L
* contraction sum_tuv D_tuv R_tuv: 2 per component
* accumulation: 1
and one point x one nucleus costs 10 (difference, R^2, Z/R, add).

The field E = -grad V (with V) of one point x one pair runs the same steps one
order further: Boys values G_0..G_{L+1}, the recursion of total order L+1,
four contractions (V and three gradient components, 2 flops per component
each) and four accumulations; one point x one nucleus costs 19 (difference 3,
R^2 5, 1/R 1, Z/R 1, Z/R^3 2, three products 3, four accumulations).
"""
from functools import lru_cache

NCOMP = (1, 4, 10, 20, 35)
NUCLEUS_FLOPS = 10
NUCLEUS_FIELD_FLOPS = 19


@lru_cache(maxsize=None)
def recursion_flops(L: int) -> int:
    total = 0
    for n in range(L - 1, -1, -1):
        m = L - n
        for t in range(m + 1):
            for u in range(m + 1 - t):
                for v in range(m + 1 - t - u):
                    if t + u + v == 0:
                        continue
                    a = t if t > 0 else (u if u > 0 else v)
                    total += 1 if a == 1 else (2 if a == 2 else 3)
    return total


@lru_cache(maxsize=None)
def pair_flops(L: int) -> int:
    return 9 + (3 * L + 4) + recursion_flops(L) + 2 * NCOMP[L] + 1


def eval_flops(n_points: int, pairs_by_L, n_nuclei: int) -> float:
    """Algorithmic flops of one evaluation at n_points points."""
    per_point = sum(int(c) * pair_flops(L) for L, c in enumerate(pairs_by_L))
    per_point += NUCLEUS_FLOPS * int(n_nuclei)
    return float(n_points) * per_point


@lru_cache(maxsize=None)
def field_pair_flops(L: int) -> int:
    return 9 + (3 * (L + 1) + 4) + recursion_flops(L + 1) + 8 * NCOMP[L] + 4


def eval_field_flops(n_points: int, pairs_by_L, n_nuclei: int) -> float:
    """Algorithmic flops of one field evaluation (V and E) at n_points points."""
    per_point = sum(int(c) * field_pair_flops(L) for L, c in enumerate(pairs_by_L))
    per_point += NUCLEUS_FIELD_FLOPS * int(n_nuclei)
    return float(n_points) * per_point

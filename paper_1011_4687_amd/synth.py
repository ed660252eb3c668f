"""Seeded synthetic QM/MM environments and QMC electron positions.

This module only draws random numbers and lays them out; it computes no
integral, normalisation, overlap or potential.  Both the product path and the
FP64 oracle consume its output, so it must stay free of the method's
arithmetic.

The environments stand in for the paper's glycine-trimer FMO-QMC benchmark
(Sec. III: the MM environment of fragment fr1; Sec. II.B, Eq.
ElectrostaticField: nuclei plus an electron density around the QM region).
That data set is not available, so every workload is synthetic with the
shape of a protein-fragment environment:

* atoms are grouped in neutral fragments of 10 (FMO fragments, Sec. II.B);
* each atom carries contracted Cartesian Gaussian shells;
* the density matrix is block diagonal per fragment, P_f = C_f C_f^T with
  Gaussian C_f (positive semidefinite, so rho >= 0 everywhere);
* QMC electron positions are uniform in the QM sphere, which no
  environment atom enters.

P_f is returned *unscaled*.  Scaling each block so that its electron count
equals the fragment's nuclear charge needs overlap integrals, which belong to
the method; the consumer applies it (the library's neutralise option, or the
oracle's overlap in tests).

Draw order inside one workload is fixed: positions -> Z -> basis -> C ->
points, from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

Z_CHOICES = np.array([1, 6, 7, 8], dtype=np.int64)


@dataclasses.dataclass
class Shell:
    atom: int            # index into the nuclei arrays (shell centre)
    l: int               # angular momentum 0, 1 or 2
    exponents: np.ndarray  # (nprim,) float64, descending
    coefs: np.ndarray      # (nprim,) float64, multiply normalised primitives


@dataclasses.dataclass
class Environment:
    """Nuclei, shells and the unscaled density blocks of one environment."""
    name: str
    xyz: np.ndarray        # (K, 3) float64, bohr
    Z: np.ndarray          # (K,) float64
    fragment: np.ndarray   # (K,) int32
    shells: List[Shell]
    # density blocks: fragment f covers basis functions [bf_lo[f], bf_hi[f])
    bf_lo: np.ndarray      # (F,) int64
    bf_hi: np.ndarray      # (F,) int64
    blocks: List[np.ndarray]  # (n_f, n_f) float64 each, C_f C_f^T (unscaled)
    r_qm: float            # radius of the QM sphere the atoms avoid

    @property
    def n_nuclei(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum(ncart(s.l) for s in self.shells))

    @property
    def n_fragments(self) -> int:
        return len(self.blocks)

    def shell_arrays(self):
        """Flat arrays: atom, l, nprim, prim_offset, exps, coefs."""
        atom = np.array([s.atom for s in self.shells], dtype=np.int32)
        l = np.array([s.l for s in self.shells], dtype=np.int32)
        nprim = np.array([len(s.exponents) for s in self.shells], dtype=np.int32)
        off = np.zeros(len(self.shells), dtype=np.int64)
        if len(self.shells):
            off[1:] = np.cumsum(nprim)[:-1]
        exps = (np.concatenate([s.exponents for s in self.shells])
                if self.shells else np.zeros(0))
        coefs = (np.concatenate([s.coefs for s in self.shells])
                 if self.shells else np.zeros(0))
        return atom, l, nprim, off, exps.astype(np.float64), coefs.astype(np.float64)

    def density_csr(self, scale: Optional[Sequence[float]] = None):
        """Block-diagonal P as CSR (row_ptr int64, col int32, val float64).

        ``scale[f]`` multiplies block f (default 1: the unscaled C_f C_f^T).
        """
        nbf = self.nbf
        row_ptr = np.zeros(nbf + 1, dtype=np.int64)
        cols, vals = [], []
        widths = np.zeros(nbf, dtype=np.int64)
        for f, blk in enumerate(self.blocks):
            lo, hi = int(self.bf_lo[f]), int(self.bf_hi[f])
            s = 1.0 if scale is None else float(scale[f])
            widths[lo:hi] = hi - lo
            for r in range(hi - lo):
                cols.append(np.arange(lo, hi, dtype=np.int32))
                vals.append(blk[r] * s)
        row_ptr[1:] = np.cumsum(widths)
        col = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int32)
        val = np.concatenate(vals) if vals else np.zeros(0)
        return row_ptr, col.astype(np.int32), val.astype(np.float64)

    def density_dense(self, scale: Optional[Sequence[float]] = None) -> np.ndarray:
        nbf = self.nbf
        P = np.zeros((nbf, nbf))
        for f, blk in enumerate(self.blocks):
            lo, hi = int(self.bf_lo[f]), int(self.bf_hi[f])
            s = 1.0 if scale is None else float(scale[f])
            P[lo:hi, lo:hi] = blk * s
        return P

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.xyz, self.Z, self.fragment, self.bf_lo, self.bf_hi):
            h.update(np.ascontiguousarray(a).tobytes())
        for s in self.shells:
            h.update(np.array([s.atom, s.l], dtype=np.int64).tobytes())
            h.update(s.exponents.tobytes())
            h.update(s.coefs.tobytes())
        for b in self.blocks:
            h.update(b.tobytes())
        return h.hexdigest()


def subset(env: Environment, fragments, name: Optional[str] = None) -> Environment:
    """The environment made of the given fragments only (their nuclei, shells
    and density blocks, in the original order).  Every fragment's block is
    kept as it is, so the fragments of a partition of an environment add up
    to the whole."""
    keep = np.zeros(env.n_fragments, dtype=bool)
    keep[np.asarray(list(fragments), dtype=np.int64)] = True
    atoms = np.nonzero(keep[env.fragment])[0]
    new_atom = -np.ones(env.n_nuclei, dtype=np.int64)
    new_atom[atoms] = np.arange(len(atoms))
    frag_ids = np.nonzero(keep)[0]
    new_frag = -np.ones(env.n_fragments, dtype=np.int64)
    new_frag[frag_ids] = np.arange(len(frag_ids))
    shells = [Shell(int(new_atom[s.atom]), s.l, s.exponents, s.coefs)
              for s in env.shells if keep[env.fragment[s.atom]]]
    bf_lo, bf_hi, blocks, o = [], [], [], 0
    for f in frag_ids:
        n = int(env.bf_hi[f] - env.bf_lo[f])
        bf_lo.append(o)
        bf_hi.append(o + n)
        blocks.append(env.blocks[f])
        o += n
    return Environment(name or f"{env.name}-subset", env.xyz[atoms].copy(), env.Z[atoms].copy(),
                       new_frag[env.fragment[atoms]].astype(np.int32), shells,
                       np.array(bf_lo, dtype=np.int64), np.array(bf_hi, dtype=np.int64), blocks, env.r_qm)


def ncart(l: int) -> int:
    """Number of Cartesian components of a shell of angular momentum l."""
    return (l + 1) * (l + 2) // 2


def _uniform_ball(u: np.ndarray, radius: float, r_min: float = 0.0) -> np.ndarray:
    """Map rows of 3 uniforms to points uniform in a ball (or shell r_min..radius)."""
    r3 = r_min ** 3 + u[:, 0] * (radius ** 3 - r_min ** 3)
    r = np.cbrt(r3)
    ct = 2.0 * u[:, 1] - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * u[:, 2]
    return np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1)


def points_in_ball(rng: np.random.Generator, n: int, radius: float,
                   r_min: float = 0.0) -> np.ndarray:
    """n points uniform in the ball |r| < radius (or the shell r_min..radius).

    Each point consumes exactly three uniforms, so the first k points do not
    depend on n.
    """
    u = rng.random((n, 3))
    return _uniform_ball(u, radius, r_min)


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def _draw_basis(rng, Z, kind):
    shells = []
    for a, z in enumerate(Z):
        if kind == "tiny":
            # 4 uncontracted s primitives + 1 uncontracted p primitive
            ls = [0, 0, 0, 0, 1]
            for l in ls:
                e = _log_uniform(rng, 0.1, 50.0, 1)
                shells.append(Shell(a, l, e.astype(np.float64), np.ones(1)))
        else:
            ls = [0, 0, 0, 1, 1, 2] if z > 1 else [0, 0, 1]
            for l in ls:
                depth = int(rng.integers(3, 7))
                e = np.sort(_log_uniform(rng, 0.05, 5000.0, depth))[::-1].copy()
                c = rng.uniform(0.1, 1.0, depth)
                shells.append(Shell(a, l, e, c))
    return shells


def _fragment_blocks(rng, shells, fragment, n_frag):
    """Per fragment: basis range and C_f C_f^T with C_f ~ N(0,1) (n_f x ceil(n_f/2))."""
    nb = np.array([ncart(s.l) for s in shells], dtype=np.int64)
    frag_of_shell = np.array([fragment[s.atom] for s in shells], dtype=np.int64)
    start = np.zeros(len(shells) + 1, dtype=np.int64)
    start[1:] = np.cumsum(nb)
    bf_lo = np.zeros(n_frag, dtype=np.int64)
    bf_hi = np.zeros(n_frag, dtype=np.int64)
    blocks = []
    for f in range(n_frag):
        idx = np.nonzero(frag_of_shell == f)[0]
        lo, hi = int(start[idx[0]]), int(start[idx[-1] + 1])
        assert np.all(np.diff(idx) == 1), "shells of a fragment must be contiguous"
        n = hi - lo
        C = rng.standard_normal((n, (n + 1) // 2))
        bf_lo[f], bf_hi[f] = lo, hi
        blocks.append(C @ C.T)
    return bf_lo, bf_hi, blocks


def _fragment_positions(rng, n_atoms, box, r_qm):
    """Fragments of 10 atoms: centre uniform in the box with |c| >= r_qm + 2,
    atoms uniform in a 3-bohr ball around it, inside the box and outside the
    QM sphere (rejection)."""
    half = box / 2.0
    xyz = np.zeros((n_atoms, 3))
    for f in range(n_atoms // 10):
        while True:
            c = rng.uniform(-half, half, 3)
            if np.linalg.norm(c) >= r_qm + 2.0:
                break
        k = 0
        while k < 10:
            a = c + _uniform_ball(rng.random((1, 3)), 3.0)[0]
            if np.linalg.norm(a) >= r_qm and np.all(np.abs(a) <= half):
                xyz[f * 10 + k] = a
                k += 1
    return xyz


def box_side(n_atoms: int) -> float:
    """Box side that keeps the 200-atom / 40-bohr atom density."""
    return 40.0 * (n_atoms / 200.0) ** (1.0 / 3.0)


def _rng(seed_or_rng):
    if isinstance(seed_or_rng, np.random.Generator):
        return seed_or_rng
    return np.random.Generator(np.random.PCG64(int(seed_or_rng)))


def make_tiny(seed=1001) -> Environment:
    """12 atoms uniform in [-8,8]^3 outside a 4-bohr sphere; Z in {1,6,7,8};
    per atom four s primitives and one p primitive (exponents log-uniform in
    [0.1, 50]); 84 basis functions; one density block C C^T, C 84 x 42.
    ``seed`` is an int or a Generator (then drawing continues on it)."""
    rng = _rng(seed)
    xyz = np.zeros((12, 3))
    k = 0
    while k < 12:
        a = rng.uniform(-8.0, 8.0, 3)
        if np.linalg.norm(a) >= 4.0:
            xyz[k] = a
            k += 1
    Z = Z_CHOICES[rng.integers(0, 4, 12)].astype(np.float64)
    shells = _draw_basis(rng, Z, "tiny")
    frag = np.zeros(12, dtype=np.int32)
    bf_lo, bf_hi, blocks = _fragment_blocks(rng, shells, frag, 1)
    return Environment("tiny", xyz, Z, frag, shells, bf_lo, bf_hi, blocks, 4.0)


def make_fragmented(n_atoms: int, seed, r_qm: float = 8.0,
                    name: str = "env") -> Environment:
    """n_atoms (a multiple of 10) in neutral 10-atom fragments in a box of side
    40 (n_atoms/200)^(1/3) bohr around an r_qm-bohr QM sphere; heavy atoms
    carry 3s/2p/1d contracted shells, H 2s/1p; depth 3..6, exponents
    log-uniform in [0.05, 5000] (descending), coefficients U(0.1, 1)."""
    assert n_atoms % 10 == 0 and n_atoms > 0
    rng = _rng(seed)
    box = box_side(n_atoms)
    xyz = _fragment_positions(rng, n_atoms, box, r_qm)
    Z = Z_CHOICES[rng.integers(0, 4, n_atoms)].astype(np.float64)
    shells = _draw_basis(rng, Z, "contracted")
    frag = (np.arange(n_atoms) // 10).astype(np.int32)
    bf_lo, bf_hi, blocks = _fragment_blocks(rng, shells, frag, n_atoms // 10)
    return Environment(name, xyz, Z, frag, shells, bf_lo, bf_hi, blocks, r_qm)


# ---------------------------------------------------------------------------
# Named workloads.  Each returns (environment, points) with a fixed seed.
# ---------------------------------------------------------------------------

WORKLOADS = {
    "tiny": dict(seed=1001, n_points=1024, r_points=4.0),
    "mid": dict(seed=1002, n_atoms=200, n_points=131072, r_points=8.0),
    "surrogate": dict(seed=1004, n_atoms=1000, n_points=1048576, r_points=6.0),
    "large": dict(seed=1005, n_atoms=5000, n_points=1048576, r_points=8.0),
}


def workload(name: str, n_points: Optional[int] = None):
    """(Environment, points[n,3]) for a named workload.

    tiny: 12 atoms, 1024 points in the 4-bohr sphere.
    mid: 200 atoms (20 fragments), 131072 points (4096 walkers x 32 electrons)
         in the 8-bohr sphere.
    surrogate: 1000 atoms, points in the 6-bohr sphere.
    large: 5000 atoms (500 fragments), 1048576 points (65536 x 16).
    """
    w = WORKLOADS[name]
    n = w["n_points"] if n_points is None else int(n_points)
    rng = _rng(w["seed"])
    if name == "tiny":
        env = make_tiny(rng)
    else:
        env = make_fragmented(w["n_atoms"], rng, 8.0, name)
    # points are the last draw, three uniforms each: the first k points do
    # not depend on n
    pts = points_in_ball(rng, n, w["r_points"])
    return env, pts


def batched_instances(n_inst: int = 64, seed0: int = 3000,
                      max_points: Optional[int] = None):
    """Uneven QM/MM instances: atoms log-uniform in [50, 2000] (rounded to a
    multiple of 10), points log-uniform in [1k, 200k]; instance i uses seed
    seed0 + i.  Returns a list of (Environment, points)."""
    out = []
    for i in range(n_inst):
        rng = _rng(seed0 + i)
        na = int(round(_log_uniform(rng, 50, 2000, 1)[0] / 10.0)) * 10
        na = max(na, 50)
        npts = int(round(_log_uniform(rng, 1000, 200000, 1)[0]))
        if max_points is not None:
            npts = min(npts, max_points)
        env = make_fragmented(na, rng, 8.0, f"inst{i}")
        out.append((env, points_in_ball(rng, npts, 8.0)))
    return out


def surrogate_sets(seed: int = 1004, n_train: int = 2_000_000,
                   n_infer: int = 1_000_000, n_out: int = 65536):
    """Point sets of the surrogate workload: training points and inference
    points uniform in the 6-bohr sphere, plus out-of-region points in the
    6..8-bohr shell that the error gate must send to the exact kernel."""
    rng = _rng(seed + 200000)
    train = points_in_ball(rng, n_train, 6.0)
    infer = points_in_ball(rng, n_infer, 6.0)
    outer = points_in_ball(rng, n_out, 8.0, r_min=6.0)
    return train, infer, outer


@dataclasses.dataclass
class CellEnvironment:
    """The paper's own form of the environment (Sec. II.B, Eq.
    ElectrostaticField): nuclei plus the electron density given on cells,
    each cell a point charge q_m = rho(r_m) h^3 (electron count, >= 0)."""
    xyz: np.ndarray      # (K, 3) nuclei, bohr
    Z: np.ndarray        # (K,)
    cells: np.ndarray    # (M, 4): x, y, z, q_m
    h: float             # cell edge, bohr

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])


def cell_workload(seed: int = 1006, n_points: int = 131072, n_atoms: int = 19,
                  h: float = 0.194, r_cut: float = 3.0, r_points: float = 3.0):
    """(CellEnvironment, points) shaped like the paper's benchmark (Sec. III:
    19 MM atoms, M = 268,782 cells, QMC electrons in the QM fragment).

    Atoms: uniform in the shell 6.5 <= |R| <= 11 bohr, at least 1.8 bohr
    apart, Z uniform in {1, 6, 7, 8}.  Cells: the points of the cubic grid of
    edge h (origin on a grid point) within r_cut of some atom; each cell
    carries a sum of atom-centred Gaussian profiles Z_A exp(-b_A d^2) with b_A
    uniform in [0.6, 1.6] 1/bohr^2, scaled so that the cells hold as many
    electrons as the nuclei carry charge (a neutral environment).  Points:
    uniform in the r_points sphere, so every point is at least 0.5 bohr from
    every cell.  Draw order: atoms -> Z -> b -> points."""
    rng = _rng(seed)
    pos = []
    while len(pos) < n_atoms:
        u = rng.uniform(-1.0, 1.0, 3)
        r = np.linalg.norm(u)
        if r == 0.0 or r > 1.0:
            continue
        c = u / r * rng.uniform(6.5, 11.0)
        if all(np.linalg.norm(c - q) >= 1.8 for q in pos):
            pos.append(c)
    xyz = np.array(pos)
    Z = Z_CHOICES[rng.integers(0, len(Z_CHOICES), n_atoms)].astype(np.float64)
    b = rng.uniform(0.6, 1.6, n_atoms)
    lo = np.floor((xyz.min(axis=0) - r_cut) / h) * h
    hi = np.ceil((xyz.max(axis=0) + r_cut) / h) * h
    axes = [np.arange(lo[k], hi[k] + 0.5 * h, h) for k in range(3)]
    gx, gy, gz = np.meshgrid(*axes, indexing="ij")
    grid = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    d2 = ((grid[:, None, :] - xyz[None, :, :]) ** 2).sum(axis=2)
    keep = (d2 <= r_cut * r_cut).any(axis=1)
    grid, d2 = grid[keep], d2[keep]
    w = (Z[None, :] * np.exp(-b[None, :] * d2)).sum(axis=1)
    q = w * (Z.sum() / w.sum())
    cells = np.concatenate([grid, q[:, None]], axis=1)
    pts = points_in_ball(rng, n_points, r_points)
    return CellEnvironment(xyz, Z, cells, h), pts


def digest(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()

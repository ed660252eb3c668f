"""Python front end of the FP64 CPU oracle (``envpot_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark are the only callers.  Nothing in the
product library imports this module.

The C file is compiled with gcc at strict IEEE settings (-O2, no fast-math,
no FMA contraction) into ``oracle/liboracle.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "envpot_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle (always when ``force``)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
        L.oracle_prim_norm.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_prim_norm.restype = ctypes.c_double
        L.oracle_overlap1d.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4
        L.oracle_overlap1d.restype = ctypes.c_double
        L.oracle_hermite_E.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 4
        L.oracle_hermite_E.restype = ctypes.c_double
        L.oracle_hermite_R.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [_dp]
        L.oracle_potential.argtypes = [
            ctypes.c_int, _dp, _dp, ctypes.c_int, _i32p, _i32p, _i32p, _i64p, _dp, _dp,
            ctypes.c_int, _i64p, _i32p, _dp, ctypes.c_int64, _dp, ctypes.c_int,
            ctypes.c_double, ctypes.c_int, _dp]
        L.oracle_potential.restype = ctypes.c_int
        L.oracle_field.argtypes = L.oracle_potential.argtypes
        L.oracle_field.restype = ctypes.c_int
        L.oracle_density_overlap_rows.argtypes = [
            ctypes.c_int, _dp, ctypes.c_int, _i32p, _i32p, _i32p, _i64p, _dp, _dp,
            ctypes.c_int, _i64p, _i32p, _dp, _dp]
        L.oracle_density_overlap_rows.restype = ctypes.c_int
        L.oracle_overlap_matrix.argtypes = [
            _dp, ctypes.c_int, _i32p, _i32p, _i32p, _i64p, _dp, _dp, ctypes.c_int, _dp]
        L.oracle_overlap_matrix.restype = ctypes.c_int
        L.oracle_count_pairs.argtypes = [
            _dp, ctypes.c_int, _i32p, _i32p, _i32p, _i64p, _dp, _dp, ctypes.c_int,
            _i64p, _i32p, _dp, ctypes.c_int, ctypes.c_double]
        L.oracle_count_pairs.restype = ctypes.c_int64
        L.oracle_set_mutation.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def set_mutation(m: int) -> None:
    lib().oracle_set_mutation(int(m))


# ------------------------------------------------------------------ pieces

def boys(nmax: int, T: float) -> np.ndarray:
    F = np.zeros(nmax + 1)
    lib().oracle_boys(int(nmax), float(T), _p(F, ctypes.c_double))
    return F


def prim_norm(a: float, i: int, j: int, k: int) -> float:
    return lib().oracle_prim_norm(float(a), i, j, k)


def overlap1d(i, j, a, b, A, B) -> float:
    return lib().oracle_overlap1d(int(i), int(j), float(a), float(b), float(A), float(B))


def hermite_E(i, j, t, a, b, A, B) -> float:
    return lib().oracle_hermite_E(int(i), int(j), int(t), float(a), float(b),
                                  float(A), float(B))


RDIM = 6


def hermite_R(L: int, p: float, X: float, Y: float, Z: float) -> np.ndarray:
    """R^0_{tuv} as an array [t, u, v] (entries with t+u+v > L are unset/0)."""
    out = np.zeros(RDIM ** 3)
    lib().oracle_hermite_R(int(L), float(p), float(X), float(Y), float(Z),
                           _p(out, ctypes.c_double))
    return out.reshape(RDIM, RDIM, RDIM)


# ---------------------------------------------------------- whole systems

class _Packed:
    def __init__(self, xyz, Z, shells_flat, P):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.Z = np.ascontiguousarray(Z, dtype=np.float64)
        atom, l, nprim, off, ex, co = shells_flat
        self.atom = np.ascontiguousarray(atom, dtype=np.int32)
        self.l = np.ascontiguousarray(l, dtype=np.int32)
        self.nprim = np.ascontiguousarray(nprim, dtype=np.int32)
        self.off = np.ascontiguousarray(off, dtype=np.int64)
        self.ex = np.ascontiguousarray(ex, dtype=np.float64)
        self.co = np.ascontiguousarray(co, dtype=np.float64)
        self.nbf = int(sum((x + 1) * (x + 2) // 2 for x in self.l))
        if P is None:
            P = (np.zeros(self.nbf + 1, dtype=np.int64), np.zeros(0, dtype=np.int32),
                 np.zeros(0))
        elif isinstance(P, np.ndarray):
            P = dense_to_csr(P)
        rowp, col, val = P
        self.rowp = np.ascontiguousarray(rowp, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        assert self.rowp.shape[0] == self.nbf + 1


def dense_to_csr(P: np.ndarray):
    P = np.asarray(P, dtype=np.float64)
    nbf = P.shape[0]
    rowp = np.zeros(nbf + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(nbf):
        nz = np.nonzero(P[i])[0]
        cols.append(nz.astype(np.int32))
        vals.append(P[i, nz])
        rowp[i + 1] = rowp[i] + len(nz)
    col = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int32)
    val = np.concatenate(vals) if vals else np.zeros(0)
    return rowp, col, val


def _pack_env(env, P=None, scale=None) -> _Packed:
    if P is None:
        P = env.density_csr(scale)
    return _Packed(env.xyz, env.Z, env.shell_arrays(), P)


def potential_raw(xyz, Z, shells_flat, P, points, screen=False, thr=1e-12,
                  nthreads=0):
    """V, V_nuc, V_ele, A at ``points`` for explicit arrays.

    shells_flat = (atom, l, nprim, prim_offset, exps, coefs); P is a dense
    matrix or a CSR triple (row_ptr, col, val) or None (no electrons)."""
    pk = _Packed(xyz, Z, shells_flat, P)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((pts.shape[0], 4))
    rc = lib().oracle_potential(
        pk.xyz.shape[0], _p(pk.xyz, ctypes.c_double), _p(pk.Z, ctypes.c_double),
        pk.l.shape[0], _p(pk.atom, ctypes.c_int32), _p(pk.l, ctypes.c_int32),
        _p(pk.nprim, ctypes.c_int32), _p(pk.off, ctypes.c_int64),
        _p(pk.ex, ctypes.c_double), _p(pk.co, ctypes.c_double), pk.nbf,
        _p(pk.rowp, ctypes.c_int64), _p(pk.col, ctypes.c_int32),
        _p(pk.val, ctypes.c_double), pts.shape[0], _p(pts, ctypes.c_double),
        int(bool(screen)), float(thr), int(nthreads), _p(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_potential: bad argument")
    return out[:, 0], out[:, 1], out[:, 2], out[:, 3]


def potential(env, points, P=None, scale=None, screen=False, thr=1e-12,
              nthreads=0):
    """V, V_nuc, V_ele, A of a synth.Environment at ``points``.

    P: explicit density (dense or CSR); default the environment's blocks,
    each multiplied by ``scale[f]``."""
    if P is None:
        P = env.density_csr(scale)
    return potential_raw(env.xyz, env.Z, env.shell_arrays(), P, points, screen,
                         thr, nthreads)


def field_raw(xyz, Z, shells_flat, P, points, screen=False, thr=1e-12, nthreads=0):
    """E = -grad V (n x 3) and the conditioning scale AE (n) at ``points``
    for explicit arrays (arguments as potential_raw)."""
    pk = _Packed(xyz, Z, shells_flat, P)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((pts.shape[0], 4))
    rc = lib().oracle_field(
        pk.xyz.shape[0], _p(pk.xyz, ctypes.c_double), _p(pk.Z, ctypes.c_double),
        pk.l.shape[0], _p(pk.atom, ctypes.c_int32), _p(pk.l, ctypes.c_int32),
        _p(pk.nprim, ctypes.c_int32), _p(pk.off, ctypes.c_int64),
        _p(pk.ex, ctypes.c_double), _p(pk.co, ctypes.c_double), pk.nbf,
        _p(pk.rowp, ctypes.c_int64), _p(pk.col, ctypes.c_int32),
        _p(pk.val, ctypes.c_double), pts.shape[0], _p(pts, ctypes.c_double),
        int(bool(screen)), float(thr), int(nthreads), _p(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_field: bad argument")
    return out[:, :3].copy(), out[:, 3].copy()


def field(env, points, P=None, scale=None, screen=False, thr=1e-12, nthreads=0):
    """E = -grad V and AE of a synth.Environment at ``points``."""
    if P is None:
        P = env.density_csr(scale)
    return field_raw(env.xyz, env.Z, env.shell_arrays(), P, points, screen, thr, nthreads)


def overlap_matrix_raw(xyz, shells_flat) -> np.ndarray:
    pk = _Packed(xyz, np.zeros(len(xyz)), shells_flat, None)
    S = np.zeros((pk.nbf, pk.nbf))
    rc = lib().oracle_overlap_matrix(
        _p(pk.xyz, ctypes.c_double), pk.l.shape[0], _p(pk.atom, ctypes.c_int32),
        _p(pk.l, ctypes.c_int32), _p(pk.nprim, ctypes.c_int32),
        _p(pk.off, ctypes.c_int64), _p(pk.ex, ctypes.c_double),
        _p(pk.co, ctypes.c_double), pk.nbf, _p(S, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_overlap_matrix: bad argument")
    return S


def overlap_matrix(env) -> np.ndarray:
    return overlap_matrix_raw(env.xyz, env.shell_arrays())


def density_overlap_rows(env, P=None, scale=None) -> np.ndarray:
    """out[mu] = sum_nu P_{mu nu} S_{mu nu}; its sum is tr(P S)."""
    pk = _pack_env(env, P, scale)
    out = np.zeros(pk.nbf)
    rc = lib().oracle_density_overlap_rows(
        pk.xyz.shape[0], _p(pk.xyz, ctypes.c_double), pk.l.shape[0],
        _p(pk.atom, ctypes.c_int32), _p(pk.l, ctypes.c_int32),
        _p(pk.nprim, ctypes.c_int32), _p(pk.off, ctypes.c_int64),
        _p(pk.ex, ctypes.c_double), _p(pk.co, ctypes.c_double), pk.nbf,
        _p(pk.rowp, ctypes.c_int64), _p(pk.col, ctypes.c_int32),
        _p(pk.val, ctypes.c_double), _p(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_density_overlap_rows: bad argument")
    return out


def fragment_electrons(env, P=None, scale=None) -> np.ndarray:
    """tr(P_f S_f) of every fragment block."""
    rows = density_overlap_rows(env, P, scale)
    return np.array([rows[int(lo):int(hi)].sum() for lo, hi in zip(env.bf_lo, env.bf_hi)])


def neutral_scales(env) -> np.ndarray:
    """s_f such that s_f tr(C_f C_f^T S_f) equals the fragment's nuclear charge."""
    q = fragment_electrons(env)
    zf = np.array([env.Z[env.fragment == f].sum() for f in range(env.n_fragments)])
    return zf / q


def count_pairs(env, screen=True, thr=1e-12, P=None) -> int:
    pk = _pack_env(env, P)
    return int(lib().oracle_count_pairs(
        _p(pk.xyz, ctypes.c_double), pk.l.shape[0], _p(pk.atom, ctypes.c_int32),
        _p(pk.l, ctypes.c_int32), _p(pk.nprim, ctypes.c_int32),
        _p(pk.off, ctypes.c_int64), _p(pk.ex, ctypes.c_double),
        _p(pk.co, ctypes.c_double), pk.nbf, _p(pk.rowp, ctypes.c_int64),
        _p(pk.col, ctypes.c_int32), _p(pk.val, ctypes.c_double), int(bool(screen)),
        float(thr)))

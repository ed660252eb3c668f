"""ctypes binding of ``libenvpot.so`` (C ABI in include/env_potential.h).

Argument marshalling only: every step of the potential runs in the library's
gfx950 kernels.  The binding refuses to work without the built library; there
is no Python or CPU fallback.

Functions with the C names take raw pointers and sizes; ``Environment`` wraps
them for numpy inputs and torch device tensors.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_uint32, c_void_p
from typing import Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libenvpot.so")

ENV_OK = 0
ENV_E_ARG = -1
ENV_E_UNSUPPORTED = -2
ENV_E_NOMEM = -3
ENV_E_DEVICE = -4
ENV_E_STATE = -5

ENV_PREC_FP64 = 0
ENV_PREC_FP32C = 1

ENV_BUILD_ONLY = 0x1
ENV_NEUTRALIZE = 0x2
ENV_NO_SCREENING = 0x4
ENV_NO_MERGE = 0x8
ENV_FORCE_CPU = 0x10
ENV_HOST_PACK = 0x20

ENV_DENSITY_DENSE = 0
ENV_DENSITY_CSR = 1

PRECISIONS = {"fp64": ENV_PREC_FP64, "fp32c": ENV_PREC_FP32C}
NCOMP = (1, 4, 10, 20, 35)


class env_nucleus(ctypes.Structure):
    _fields_ = [("xyz", c_double * 3), ("Z", c_double), ("fragment", c_int32),
                ("reserved", c_int32)]


class env_shell(ctypes.Structure):
    _fields_ = [("atom", c_int32), ("l", c_int32), ("nprim", c_int32), ("reserved", c_int32),
                ("exponents", POINTER(c_double)), ("coefs", POINTER(c_double))]


class env_density(ctypes.Structure):
    _fields_ = [("nbf", c_int32), ("format", c_int32), ("values", POINTER(c_double)),
                ("row_ptr", POINTER(c_int64)), ("col", POINTER(c_int32))]


class env_options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("device", c_int32), ("screen_threshold", c_double),
                ("flags", c_uint32), ("reserved", c_int32 * 3)]


class env_peak(ctypes.Structure):
    _fields_ = [("fp32_fma_tflops", c_double), ("fp64_fma_tflops", c_double),
                ("rsq_f32_per_s", c_double), ("ms", c_double * 3)]


class env_info(ctypes.Structure):
    _fields_ = [("nbf", c_int32), ("n_nuclei", c_int32), ("n_groups", c_int32),
                ("n_segments", c_int32), ("n_pairs", c_int64), ("n_pairs_by_L", c_int64 * 5),
                ("n_pairs_unscreened", c_int64), ("electrons", c_double),
                ("nuclear_charge", c_double), ("screened_bound", c_double),
                ("device_bytes", c_int64), ("precision", c_int32),
                ("built_on_device", c_int32), ("n_clusters", c_int64),
                ("n_cluster_members", c_int64), ("on_host", c_int32), ("pairs_built_on_device", c_int32)]


class env_batch_stats(ctypes.Structure):
    _fields_ = [("n_items", c_int64), ("grid", c_int32), ("np", c_int32),
                ("launches", c_int64), ("captures", c_int64), ("graph_launches", c_int64),
                ("granularity", c_int32), ("reserved", c_int32), ("sorted_points", c_int64),
                ("sorts", c_int64), ("autotunes", c_int64)]


class env_server_stats(ctypes.Structure):
    _fields_ = [("rounds", c_int64), ("requests", c_int64), ("points", c_int64), ("errors", c_int64),
                ("busy_seconds", c_double), ("clients", c_int32), ("reserved", c_int32)]


class env_surrogate_spec(ctypes.Structure):
    _fields_ = [("n_freq", c_int32), ("hidden", c_int32), ("layers", c_int32),
                ("poly_degree", c_int32), ("radius", c_double), ("B", POINTER(c_double)),
                ("params", POINTER(ctypes.c_float)), ("poly", POINTER(c_double)),
                ("sigma", c_double), ("reserved", c_int32 * 4)]


class env_train_opts(ctypes.Structure):
    _fields_ = [("n_train", c_int64), ("epochs", c_int32), ("batch", c_int32), ("lr", c_double),
                ("lr_final", c_double), ("seed", ctypes.c_uint64), ("gate_grid", c_int32),
                ("gate_samples", c_int32), ("gate_tol", c_double), ("n_fit", c_int64),
                ("poly_degree", c_int32), ("reserved", c_int32 * 3)]


class env_surrogate_info(ctypes.Structure):
    _fields_ = [("n_params", c_int64), ("n_freq", c_int32), ("hidden", c_int32),
                ("layers", c_int32), ("poly_degree", c_int32), ("radius", c_double),
                ("sigma", c_double), ("baseline_rms", c_double), ("train_steps", c_int64),
                ("final_loss", c_double), ("epoch_loss", c_double * 64),
                ("teacher_seconds", c_double), ("train_seconds", c_double),
                ("gate_seconds", c_double), ("gate_grid", c_int32), ("reserved0", c_int32),
                ("gate_voxels_in_ball", c_int64), ("gate_voxels_pass", c_int64),
                ("gate_pass_volume_fraction", c_double), ("gate_max_err_passed", c_double),
                ("gate_tol", c_double), ("last_eval_n", c_int64), ("last_eval_fallback", c_int64)]


class env_surrogate_trace(ctypes.Structure):
    _fields_ = [("H", POINTER(ctypes.c_float)), ("Z", POINTER(ctypes.c_float)), ("y", POINTER(ctypes.c_float)),
                ("dy", POINTER(ctypes.c_float)), ("dH", POINTER(ctypes.c_float)), ("dZ", POINTER(ctypes.c_float)),
                ("grad", POINTER(ctypes.c_float)), ("loss", c_double)]


class EnvError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {env_status_string(status)} ({status})")


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run paper_1011_4687_amd.build.build() "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.env_options_default.argtypes = [POINTER(env_options)]
        L.env_options_default.restype = None
        L.env_status_string.argtypes = [c_int32]
        L.env_status_string.restype = ctypes.c_char_p
        L.env_potential_create.argtypes = [POINTER(env_nucleus), c_int32, POINTER(env_shell),
                                           c_int32, POINTER(env_density), POINTER(env_options),
                                           POINTER(c_void_p)]
        L.env_potential_create.restype = c_int32
        L.env_potential_eval.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
        L.env_potential_eval.restype = c_int32
        L.env_potential_eval_noalloc.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
        L.env_potential_eval_noalloc.restype = c_int32
        L.env_potential_noalloc_max_points.argtypes = []
        L.env_potential_noalloc_max_points.restype = c_int64
        L.env_potential_eval_field.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
        L.env_potential_eval_field.restype = c_int32
        L.env_potential_update_density.argtypes = [c_void_p, POINTER(env_density), c_void_p]
        L.env_potential_update_density.restype = c_int32
        L.env_potential_eval_batched.argtypes = [POINTER(c_void_p), c_int32, POINTER(c_void_p),
                                                 POINTER(c_int64), POINTER(c_void_p), c_void_p]
        L.env_potential_eval_batched.restype = c_int32
        L.env_peak_probe.argtypes = [c_int32, POINTER(env_peak)]
        L.env_peak_probe.restype = c_int32
        L.env_potential_info.argtypes = [c_void_p, POINTER(env_info)]
        L.env_potential_info.restype = c_int32
        L.env_potential_export_pairs.argtypes = [c_void_p, c_int64, POINTER(c_int32),
                                                 POINTER(c_int32), POINTER(c_double),
                                                 POINTER(c_double), POINTER(c_double)]
        L.env_potential_export_pairs.restype = c_int32
        L.env_potential_export_image.argtypes = [c_void_p, POINTER(c_uint32), c_int64, POINTER(c_int64),
                                                 POINTER(c_uint32), c_int64, POINTER(c_int64)]
        L.env_potential_export_image.restype = c_int32
        L.env_potential_destroy.argtypes = [c_void_p]
        L.env_potential_destroy.restype = None
        L.env_potential_autotune.argtypes = [c_void_p, c_void_p, c_int64, c_void_p]
        L.env_potential_autotune.restype = c_int32
        L.env_potential_kernel_timing.argtypes = [c_void_p, c_int32]
        L.env_potential_kernel_timing.restype = c_int32
        L.env_potential_kernel_times.argtypes = [c_void_p, POINTER(ctypes.c_float), c_int32, POINTER(c_int32)]
        L.env_potential_kernel_times.restype = c_int32
        L.env_batch_create.argtypes = [POINTER(c_void_p), c_int32, POINTER(c_void_p)]
        L.env_batch_create.restype = c_int32
        L.env_batch_eval.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_int64),
                                     POINTER(c_void_p), c_void_p]
        L.env_batch_eval.restype = c_int32
        L.env_batch_autotune.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_int64),
                                         POINTER(c_void_p), c_void_p]
        L.env_batch_autotune.restype = c_int32
        L.env_batch_get_stats.argtypes = [c_void_p, POINTER(env_batch_stats)]
        L.env_batch_get_stats.restype = c_int32
        L.env_batch_destroy.argtypes = [c_void_p]
        L.env_batch_destroy.restype = None
        L.env_train_opts_default.argtypes = [POINTER(env_train_opts)]
        L.env_train_opts_default.restype = None
        L.env_surrogate_create.argtypes = [c_void_p, POINTER(env_surrogate_spec), POINTER(c_void_p)]
        L.env_surrogate_create.restype = c_int32
        L.env_surrogate_train.argtypes = [c_void_p, c_void_p, POINTER(env_train_opts), c_void_p]
        L.env_surrogate_train.restype = c_int32
        L.env_surrogate_predict.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
        L.env_surrogate_predict.restype = c_int32
        L.env_surrogate_eval.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
        L.env_surrogate_eval.restype = c_int32
        L.env_surrogate_loss_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_int64,
                                              POINTER(ctypes.c_float), POINTER(c_double), c_void_p]
        L.env_surrogate_loss_grad.restype = c_int32
        L.env_surrogate_set_near.argtypes = [c_void_p, c_void_p]
        L.env_surrogate_set_near.restype = c_int32
        L.env_surrogate_trace_step.argtypes = [c_void_p, c_void_p, c_void_p, c_int64,
                                               POINTER(env_surrogate_trace), c_void_p]
        L.env_surrogate_trace_step.restype = c_int32
        L.env_surrogate_get_params.argtypes = [c_void_p, POINTER(ctypes.c_float), POINTER(c_double),
                                               POINTER(c_double)]
        L.env_surrogate_get_params.restype = c_int32
        L.env_surrogate_get_info.argtypes = [c_void_p, POINTER(env_surrogate_info)]
        L.env_surrogate_get_info.restype = c_int32
        L.env_surrogate_destroy.argtypes = [c_void_p]
        L.env_surrogate_destroy.restype = None
        L.env_cells_create.argtypes = [POINTER(env_nucleus), c_int32, POINTER(c_double), c_int64,
                                       POINTER(env_options), POINTER(c_void_p)]
        L.env_cells_create.restype = c_int32
        L.env_cells_eval.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
        L.env_cells_eval.restype = c_int32
        L.env_cells_eval_single.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
        L.env_cells_eval_single.restype = c_int32
        L.env_cells_resident_start.argtypes = [c_void_p, c_int32, c_double]
        L.env_cells_resident_start.restype = c_int32
        L.env_cells_resident_eval.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double), c_double]
        L.env_cells_resident_eval.restype = c_int32
        L.env_cells_resident_stop.argtypes = [c_void_p]
        L.env_cells_resident_stop.restype = c_int32
        L.env_cells_destroy.argtypes = [c_void_p]
        L.env_cells_destroy.restype = None
        L.env_server_create.argtypes = [POINTER(c_void_p), c_int32, ctypes.c_char_p, c_int32, c_int64,
                                        c_int32, POINTER(c_void_p)]
        L.env_server_create.restype = c_int32
        L.env_server_get_stats.argtypes = [c_void_p, POINTER(env_server_stats)]
        L.env_server_get_stats.restype = c_int32
        L.env_server_destroy.argtypes = [c_void_p]
        L.env_server_destroy.restype = None
        L.env_client_attach.argtypes = [ctypes.c_char_p, POINTER(c_void_p)]
        L.env_client_attach.restype = c_int32
        L.env_client_info.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int64), POINTER(c_int32)]
        L.env_client_info.restype = c_int32
        L.env_client_eval.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_int32]
        L.env_client_eval.restype = c_int32
        L.env_client_detach.argtypes = [c_void_p]
        L.env_client_detach.restype = None
        _lib = L
    return _lib


# ------------------------------------------------------------ C-named calls

def env_status_string(status: int) -> str:
    return lib().env_status_string(int(status)).decode()


def env_options_default() -> env_options:
    o = env_options()
    lib().env_options_default(ctypes.byref(o))
    return o


def env_potential_create(nuclei, n_nuclei, shells, n_shells, density, options) -> int:
    """Returns the handle (an integer address); raises EnvError on failure."""
    h = c_void_p()
    st = lib().env_potential_create(nuclei, int(n_nuclei), shells, int(n_shells),
                                    ctypes.byref(density), ctypes.byref(options),
                                    ctypes.byref(h))
    if st != ENV_OK:
        raise EnvError(st, "env_potential_create")
    return h.value


def env_potential_eval(handle: int, points_ptr: int, n: int, out_ptr: int,
                       stream: int = 0) -> None:
    st = lib().env_potential_eval(c_void_p(handle), c_void_p(points_ptr), int(n),
                                  c_void_p(out_ptr), c_void_p(stream))
    if st != ENV_OK:
        raise EnvError(st, "env_potential_eval")


def env_potential_eval_noalloc(handle: int, points_ptr: int, n: int, out_ptr: int,
                               stream: int = 0) -> None:
    st = lib().env_potential_eval_noalloc(c_void_p(handle), c_void_p(points_ptr), int(n),
                                          c_void_p(out_ptr), c_void_p(stream))
    if st != ENV_OK:
        raise EnvError(st, "env_potential_eval_noalloc")


def env_potential_noalloc_max_points() -> int:
    return int(lib().env_potential_noalloc_max_points())


def env_potential_eval_field(handle: int, points_ptr: int, n: int, out_ptr: int,
                             stream: int = 0) -> None:
    st = lib().env_potential_eval_field(c_void_p(handle), c_void_p(points_ptr), int(n),
                                        c_void_p(out_ptr), c_void_p(stream))
    if st != ENV_OK:
        raise EnvError(st, "env_potential_eval_field")


def env_potential_eval_batched(handles: Sequence[int], points_ptrs: Sequence[int],
                               ns: Sequence[int], out_ptrs: Sequence[int],
                               stream: int = 0) -> None:
    k = len(handles)
    H = (c_void_p * k)(*handles)
    Pp = (c_void_p * k)(*points_ptrs)
    N = (c_int64 * k)(*[int(x) for x in ns])
    O = (c_void_p * k)(*out_ptrs)
    st = lib().env_potential_eval_batched(H, k, Pp, N, O, c_void_p(stream))
    if st != ENV_OK:
        raise EnvError(st, "env_potential_eval_batched")


def env_potential_autotune(handle: int, points_ptr: int, n: int, stream: int = 0) -> None:
    st = lib().env_potential_autotune(c_void_p(handle), c_void_p(points_ptr), int(n),
                                      c_void_p(stream))
    if st != ENV_OK:
        raise EnvError(st, "env_potential_autotune")


def env_batch_create(handles: Sequence[int]) -> int:
    k = len(handles)
    H = (c_void_p * k)(*handles)
    b = c_void_p()
    st = lib().env_batch_create(H, k, ctypes.byref(b))
    if st != ENV_OK:
        raise EnvError(st, "env_batch_create")
    return b.value


def env_batch_eval(batch: int, points_ptrs: Sequence[int], ns: Sequence[int],
                   out_ptrs: Sequence[int], stream: int = 0) -> None:
    k = len(points_ptrs)
    Pp = (c_void_p * k)(*points_ptrs)
    N = (c_int64 * k)(*[int(x) for x in ns])
    O = (c_void_p * k)(*out_ptrs)
    st = lib().env_batch_eval(c_void_p(batch), Pp, N, O, c_void_p(stream))
    if st != ENV_OK:
        raise EnvError(st, "env_batch_eval")


def env_batch_get_stats(batch: int) -> dict:
    s = env_batch_stats()
    st = lib().env_batch_get_stats(c_void_p(batch), ctypes.byref(s))
    if st != ENV_OK:
        raise EnvError(st, "env_batch_get_stats")
    return {f: getattr(s, f) for f, _ in env_batch_stats._fields_}


def env_batch_destroy(batch: int) -> None:
    if batch:
        lib().env_batch_destroy(c_void_p(batch))


def peak_probe(device: int = -1) -> dict:
    """Vector-ALU rates the device sustains (independent FMA / rsq streams)."""
    r = env_peak()
    st = lib().env_peak_probe(int(device), ctypes.byref(r))
    if st != ENV_OK:
        raise EnvError(st, "env_peak_probe")
    return {"fp32_fma_tflops": r.fp32_fma_tflops, "fp64_fma_tflops": r.fp64_fma_tflops,
            "rsq_f32_per_s": r.rsq_f32_per_s, "ms": list(r.ms)}


def env_potential_info(handle: int) -> env_info:
    info = env_info()
    st = lib().env_potential_info(c_void_p(handle), ctypes.byref(info))
    if st != ENV_OK:
        raise EnvError(st, "env_potential_info")
    return info


def env_potential_destroy(handle: int) -> None:
    if handle:
        lib().env_potential_destroy(c_void_p(handle))


# -------------------------------------------------------------- wrapper

def _dp(a):
    return a.ctypes.data_as(POINTER(c_double))


class Environment:
    """One environment uploaded to the device (or built on the host only).

    xyz (K,3), Z (K,), fragment (K,) describe the nuclei; shells is a list of
    (atom, l, exponents, coefs); P is a dense (nbf,nbf) array or a CSR
    triple (row_ptr, col, values)."""

    def __init__(self, xyz, Z, fragment, shells, P, precision: str = "fp32c",
                 device: int = -1, screen_threshold: float = 1e-12,
                 neutralize: bool = False, build_only: bool = False,
                 screening: bool = True, merge: bool = True, force_cpu: bool = False,
                 host_pack: bool = False):
        self.handle = 0
        self.on_host = bool(force_cpu)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        K = xyz.shape[0]
        Z = np.ascontiguousarray(Z, dtype=np.float64).reshape(K)
        frag = np.ascontiguousarray(fragment, dtype=np.int32).reshape(K)
        nuc = (env_nucleus * max(K, 1))()
        for a in range(K):
            nuc[a].xyz[0], nuc[a].xyz[1], nuc[a].xyz[2] = xyz[a]
            nuc[a].Z = Z[a]
            nuc[a].fragment = int(frag[a])
        self._keep = []
        sh = (env_shell * max(len(shells), 1))()
        for s, (atom, l, ex, co) in enumerate(shells):
            ex = np.ascontiguousarray(ex, dtype=np.float64)
            co = np.ascontiguousarray(co, dtype=np.float64)
            self._keep += [ex, co]
            sh[s].atom, sh[s].l, sh[s].nprim = int(atom), int(l), int(ex.shape[0])
            sh[s].exponents, sh[s].coefs = _dp(ex), _dp(co)
        nbf = int(sum((l + 1) * (l + 2) // 2 for (_, l, _, _) in shells))
        self.nbf = nbf
        dens = _density(P, nbf, self._keep)
        opt = env_options_default()
        opt.precision = PRECISIONS[precision]
        opt.device = int(device)
        opt.screen_threshold = float(screen_threshold)
        opt.flags = ((ENV_NEUTRALIZE if neutralize else 0) | (ENV_BUILD_ONLY if build_only else 0)
                     | (0 if screening else ENV_NO_SCREENING) | (0 if merge else ENV_NO_MERGE)
                     | (ENV_FORCE_CPU if force_cpu else 0) | (ENV_HOST_PACK if host_pack else 0))
        self.precision = precision
        self.handle = env_potential_create(nuc, K, sh, len(shells), dens, opt)
        self._keep = None

    def update_density(self, P, stream=None):
        """Replace the density matrix (same nbf, no new nonzero blocks): the
        device refolds every pair's Hermite density in place."""
        keep = []
        dens = _density(P, self.nbf, keep)
        s = 0
        if stream is not None:
            s = stream.cuda_stream
        else:
            try:
                import torch
                s = torch.cuda.current_stream().cuda_stream
            except Exception:
                s = 0
        st = lib().env_potential_update_density(c_void_p(self.handle), ctypes.byref(dens), c_void_p(s))
        if st != ENV_OK:
            raise EnvError(st, "env_potential_update_density")

    @classmethod
    def from_synth(cls, env, scale=None, **kw) -> "Environment":
        shells = [(s.atom, s.l, s.exponents, s.coefs) for s in env.shells]
        return cls(env.xyz, env.Z, env.fragment, shells, env.density_csr(scale), **kw)

    def info(self) -> dict:
        i = env_potential_info(self.handle)
        d = {f: getattr(i, f) for f, _ in env_info._fields_}
        d["n_pairs_by_L"] = list(i.n_pairs_by_L)
        return d

    def export_pairs(self):
        """(L, group, center[n,3], p, D[n,35]) of a build-only handle."""
        n = self.info()["n_pairs"]
        L = np.zeros(max(n, 1), dtype=np.int32)
        g = np.zeros(max(n, 1), dtype=np.int32)
        c = np.zeros((max(n, 1), 3))
        p = np.zeros(max(n, 1))
        D = np.zeros((max(n, 1), 35))
        st = lib().env_potential_export_pairs(
            c_void_p(self.handle), max(n, 1), L.ctypes.data_as(POINTER(c_int32)),
            g.ctypes.data_as(POINTER(c_int32)), _dp(c), _dp(p), _dp(D))
        if st != ENV_OK:
            raise EnvError(st, "env_potential_export_pairs")
        return L[:n], g[:n], c[:n], p[:n], D[:n]

    def export_image(self):
        """(records, segments) of a device handle as uint32 arrays: the record
        words and the segment tables of every split factor (8 words each)."""
        rw, sw = c_int64(0), c_int64(0)
        h = c_void_p(self.handle)
        st = lib().env_potential_export_image(h, None, 0, ctypes.byref(rw), None, 0, ctypes.byref(sw))
        if st != ENV_OK:
            raise EnvError(st, "env_potential_export_image")
        rec = np.zeros(max(rw.value, 1), dtype=np.uint32)
        seg = np.zeros(max(sw.value, 1), dtype=np.uint32)
        st = lib().env_potential_export_image(h, rec.ctypes.data_as(POINTER(c_uint32)), rec.size, ctypes.byref(rw),
                                              seg.ctypes.data_as(POINTER(c_uint32)), seg.size, ctypes.byref(sw))
        if st != ENV_OK:
            raise EnvError(st, "env_potential_export_image")
        return rec[:rw.value], seg[:sw.value]

    def eval_host(self, points) -> np.ndarray:
        """V at (n,3) host points of a handle built with force_cpu=True
        (ENV_FORCE_CPU: the library's host threads, FP64); numpy in and out."""
        if not self.on_host:
            raise TypeError("eval_host needs a handle created with force_cpu=True")
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        out = np.empty(pts.shape[0])
        env_potential_eval(self.handle, pts.ctypes.data, pts.shape[0], out.ctypes.data, 0)
        return out

    def eval(self, points, out=None, stream=None):
        """V at a (n,3) float64 torch CUDA tensor; returns a (n,) tensor."""
        import torch
        if self.on_host:
            raise TypeError("a force_cpu handle evaluates host arrays: use eval_host")
        if not (isinstance(points, torch.Tensor) and points.is_cuda):
            raise TypeError("points must be a torch CUDA tensor")
        if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3:
            raise TypeError("points must be float64 of shape (n, 3)")
        points = points.contiguous()
        n = points.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=points.device)
        if out.dtype != torch.float64 or out.numel() != n or not out.is_contiguous():
            raise TypeError("out must be a contiguous float64 tensor of n elements")
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        env_potential_eval(self.handle, points.data_ptr(), n, out.data_ptr(),
                           stream.cuda_stream)
        return out

    def eval_noalloc(self, points, out, stream=None):
        """env_potential_eval_noalloc: V at a (n,3) float64 CUDA tensor into the
        caller's (n,) float64 tensor `out`, with no device allocation."""
        import torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda and points.is_contiguous()):
            raise TypeError("points must be a contiguous torch CUDA tensor")
        if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3:
            raise TypeError("points must be float64 of shape (n, 3)")
        n = points.shape[0]
        if out.dtype != torch.float64 or out.numel() != n or not out.is_contiguous():
            raise TypeError("out must be a contiguous float64 tensor of n elements")
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        env_potential_eval_noalloc(self.handle, points.data_ptr(), n, out.data_ptr(), stream.cuda_stream)
        return out

    def eval_field(self, points, out=None, stream=None):
        """V and the field E = -grad V at a (n,3) float64 torch CUDA tensor;
        returns a (n,4) tensor of rows (V, E_x, E_y, E_z)."""
        import torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda):
            raise TypeError("points must be a torch CUDA tensor")
        if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3:
            raise TypeError("points must be float64 of shape (n, 3)")
        points = points.contiguous()
        n = points.shape[0]
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float64, device=points.device)
        if out.dtype != torch.float64 or out.numel() != 4 * n or not out.is_contiguous():
            raise TypeError("out must be a contiguous float64 tensor of n x 4 elements")
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        env_potential_eval_field(self.handle, points.data_ptr(), n, out.data_ptr(),
                                 stream.cuda_stream)
        return out

    def kernel_timing(self, on: bool = True):
        """Record HIP events around every later potential-kernel launch."""
        _check(lib().env_potential_kernel_timing(c_void_p(self.handle), int(bool(on))),
               "env_potential_kernel_timing")

    def kernel_times(self) -> list:
        """Durations (ms) of the potential-kernel launches recorded so far."""
        cnt = c_int32()
        _check(lib().env_potential_kernel_times(c_void_p(self.handle), None, 0, ctypes.byref(cnt)),
               "env_potential_kernel_times")
        ms = (ctypes.c_float * max(cnt.value, 1))()
        _check(lib().env_potential_kernel_times(c_void_p(self.handle), ms, cnt.value, ctypes.byref(cnt)),
               "env_potential_kernel_times")
        return [float(ms[i]) for i in range(cnt.value)]

    def autotune(self, points, stream=None):
        """Time the launch shapes at these (n,3) device points; keep the best."""
        import torch
        points = points.contiguous()
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        env_potential_autotune(self.handle, points.data_ptr(), points.shape[0], stream.cuda_stream)

    def close(self):
        if self.handle:
            env_potential_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A persistent-launch plan over several Environments (same precision)."""

    def __init__(self, envs: Sequence[Environment]):
        self.envs = list(envs)
        self.handle = env_batch_create([e.handle for e in self.envs])

    def eval(self, points: Sequence, outs: Optional[Sequence] = None, stream=None):
        import torch
        if outs is None:
            outs = [torch.empty(p.shape[0], dtype=torch.float64, device=p.device) for p in points]
        if stream is None:
            stream = torch.cuda.current_stream()
        for p, o in zip(points, outs):
            if p.dtype != torch.float64 or not p.is_contiguous() or p.dim() != 2 or p.shape[1] != 3:
                raise TypeError("points must be contiguous float64 (n, 3) tensors")
            if o.dtype != torch.float64 or not o.is_contiguous() or o.numel() != p.shape[0]:
                raise TypeError("out must be contiguous float64 tensors of n elements")
        env_batch_eval(self.handle, [p.data_ptr() for p in points], [p.shape[0] for p in points],
                       [o.data_ptr() for o in outs], stream.cuda_stream)
        return outs

    def autotune(self, points: Sequence, outs: Sequence, stream=None):
        """env_batch_autotune: time the plan's launch shapes on these buffers
        and keep the fastest (synchronous; writes outs)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        n = len(points)
        pp = (c_void_p * n)(*[p.data_ptr() for p in points])
        nn = (c_int64 * n)(*[p.shape[0] for p in points])
        oo = (c_void_p * n)(*[o.data_ptr() for o in outs])
        _check(lib().env_batch_autotune(c_void_p(self.handle), pp, nn, oo, c_void_p(stream.cuda_stream)),
               "env_batch_autotune")
        return outs

    def stats(self) -> dict:
        return env_batch_get_stats(self.handle)

    def close(self):
        if self.handle:
            env_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


N_SURROGATE_PARAMS = 4 * (128 * 128 + 128) + 128 + 1


def _check(st, what):
    if st != ENV_OK:
        raise EnvError(st, what)


class Surrogate:
    """Coordinate-MLP surrogate with a validated voxel gate (env_surrogate_*).

    fallback: Environment evaluated for gated-out points; B: (64, 3)
    frequencies; params: initial parameter vector (66,177 float32)."""

    def __init__(self, fallback: Environment, B, params, radius: float = 6.0,
                 poly_degree: int = 0, poly=None, sigma: float = 1.0):
        self.fallback = fallback
        self._B = np.ascontiguousarray(B, dtype=np.float64).reshape(64, 3)
        self._p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if self._p.shape[0] != N_SURROGATE_PARAMS:
            raise ValueError("params must hold 66,177 values")
        spec = env_surrogate_spec()
        spec.n_freq, spec.hidden, spec.layers, spec.poly_degree = 64, 128, 4, int(poly_degree)
        spec.radius = float(radius)
        spec.B = _dp(self._B)
        spec.params = self._p.ctypes.data_as(POINTER(ctypes.c_float))
        if poly is not None:
            self._poly = np.ascontiguousarray(poly, dtype=np.float64)
            spec.poly = _dp(self._poly)
        spec.sigma = float(sigma)
        h = c_void_p()
        _check(lib().env_surrogate_create(c_void_p(fallback.handle), ctypes.byref(spec),
                                          ctypes.byref(h)), "env_surrogate_create")
        self.handle = h.value
        self.radius = radius
        self.near = None

    def set_near(self, near: Optional[Environment]):
        """Exact part added to the network (env_surrogate_set_near): the
        handle of the fragments the network does not cover, or None."""
        _check(lib().env_surrogate_set_near(c_void_p(self.handle), c_void_p(near.handle if near else None)),
               "env_surrogate_set_near")
        self.near = near

    @staticmethod
    def default_opts(**kw) -> env_train_opts:
        o = env_train_opts()
        lib().env_train_opts_default(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def train(self, teacher: Environment, stream=None, **kw):
        import torch
        o = self.default_opts(**kw)
        st = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().env_surrogate_train(c_void_p(self.handle), c_void_p(teacher.handle),
                                         ctypes.byref(o), c_void_p(st)), "env_surrogate_train")

    def predict(self, points, stream=None, out=None):
        """Network + baseline (no gate, no exact part) at (n,3) float64
        device points."""
        import torch
        points = points.contiguous()
        if out is None:
            out = torch.empty(points.shape[0], dtype=torch.float64, device=points.device)
        st = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().env_surrogate_predict(c_void_p(self.handle), c_void_p(points.data_ptr()),
                                           points.shape[0], c_void_p(out.data_ptr()), c_void_p(st)),
               "env_surrogate_predict")
        return out

    def eval(self, points, stream=None, out=None, used=None):
        """(V, used_fallback) at (n,3) float64 device points; asynchronous."""
        import torch
        points = points.contiguous()
        n = points.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=points.device)
        if used is None:
            used = torch.empty(n, dtype=torch.uint8, device=points.device)
        if out.dtype != torch.float64 or out.numel() != n or used.dtype != torch.uint8 or used.numel() != n:
            raise TypeError("out must be float64 and used uint8, n elements each")
        st = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().env_surrogate_eval(c_void_p(self.handle), c_void_p(points.data_ptr()), n,
                                        c_void_p(out.data_ptr()), c_void_p(used.data_ptr()),
                                        c_void_p(st)), "env_surrogate_eval")
        return out, used

    def loss_grad(self, points, targets, stream=None):
        import torch
        points = points.contiguous()
        targets = targets.to(torch.float32).contiguous()
        g = np.zeros(N_SURROGATE_PARAMS, dtype=np.float32)
        loss = c_double()
        st = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().env_surrogate_loss_grad(c_void_p(self.handle), c_void_p(points.data_ptr()),
                                             c_void_p(targets.data_ptr()), points.shape[0],
                                             g.ctypes.data_as(POINTER(ctypes.c_float)),
                                             ctypes.byref(loss), c_void_p(st)),
               "env_surrogate_loss_grad")
        return loss.value, g

    def trace_step(self, points, targets, stream=None) -> dict:
        """One forward/backward pass with every intermediate tensor copied out
        (env_surrogate_trace_step): H (5,n,128), Z (4,n,128), y, dy, dH
        (4,n,128), dZ (4,n,128), grad, loss."""
        import torch
        points = points.contiguous()
        targets = targets.to(torch.float32).contiguous()
        n = points.shape[0]
        out = {"H": np.zeros((5, n, 128), np.float32), "Z": np.zeros((4, n, 128), np.float32),
               "y": np.zeros(n, np.float32), "dy": np.zeros(n, np.float32),
               "dH": np.zeros((4, n, 128), np.float32), "dZ": np.zeros((4, n, 128), np.float32),
               "grad": np.zeros(N_SURROGATE_PARAMS, np.float32)}
        tr = env_surrogate_trace()
        for k in ("H", "Z", "y", "dy", "dH", "dZ", "grad"):
            setattr(tr, k, out[k].ctypes.data_as(POINTER(ctypes.c_float)))
        st = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().env_surrogate_trace_step(c_void_p(self.handle), c_void_p(points.data_ptr()),
                                              c_void_p(targets.data_ptr()), n, ctypes.byref(tr), c_void_p(st)),
               "env_surrogate_trace_step")
        out["loss"] = tr.loss
        return out

    def params(self):
        p = np.zeros(N_SURROGATE_PARAMS, dtype=np.float32)
        poly = np.zeros(165)
        sig = c_double()
        _check(lib().env_surrogate_get_params(c_void_p(self.handle),
                                              p.ctypes.data_as(POINTER(ctypes.c_float)),
                                              _dp(poly), ctypes.byref(sig)),
               "env_surrogate_get_params")
        return p, poly, sig.value

    def info(self) -> dict:
        i = env_surrogate_info()
        _check(lib().env_surrogate_get_info(c_void_p(self.handle), ctypes.byref(i)),
               "env_surrogate_get_info")
        d = {f: getattr(i, f) for f, _ in env_surrogate_info._fields_}
        d["epoch_loss"] = list(i.epoch_loss)
        return d

    def close(self):
        if self.handle:
            lib().env_surrogate_destroy(c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CellEnvironment:
    """The paper's own form of the environment: nuclei plus M point-charge
    cells (xyz (K,3), Z (K,), cells (M,4): x, y, z, electron count)."""

    def __init__(self, xyz, Z, cells, precision: str = "fp32c", device: int = -1):
        self.handle = 0
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        K = xyz.shape[0]
        Z = np.ascontiguousarray(Z, dtype=np.float64).reshape(K)
        nuc = (env_nucleus * max(K, 1))()
        for a in range(K):
            nuc[a].xyz[0], nuc[a].xyz[1], nuc[a].xyz[2] = xyz[a]
            nuc[a].Z = Z[a]
        c = np.ascontiguousarray(cells, dtype=np.float64).reshape(-1, 4)
        opt = env_options_default()
        opt.precision = PRECISIONS[precision]
        opt.device = int(device)
        h = c_void_p()
        _check(lib().env_cells_create(nuc, K, _dp(c), c.shape[0], ctypes.byref(opt), ctypes.byref(h)),
               "env_cells_create")
        self.handle = h.value
        self.precision = precision
        self.n_cells = c.shape[0]

    @classmethod
    def from_synth(cls, env, **kw) -> "CellEnvironment":
        return cls(env.xyz, env.Z, env.cells, **kw)

    def eval(self, points, out=None, stream=None):
        """V at a (n,3) float64 CUDA tensor; returns a (n,) tensor."""
        import torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda):
            raise TypeError("points must be a torch CUDA tensor")
        if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3:
            raise TypeError("points must be float64 of shape (n, 3)")
        points = points.contiguous()
        n = points.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=points.device)
        if out.dtype != torch.float64 or out.numel() != n or not out.is_contiguous():
            raise TypeError("out must be a contiguous float64 tensor of n elements")
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().env_cells_eval(c_void_p(self.handle), c_void_p(points.data_ptr()), n,
                                    c_void_p(out.data_ptr()), c_void_p(stream.cuda_stream)),
               "env_cells_eval")
        return out

    def eval_single(self, point, out, mode: int = 0, stream=None):
        """V at one device point (3 float64) into out (1 float64, device):
        mode 0 fills the GPU, mode 1 is the paper's 120 x 256 decomposition."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        if point.dtype != torch.float64 or point.numel() != 3 or not point.is_cuda:
            raise TypeError("point must be 3 float64 values on the device")
        if out.dtype != torch.float64 or out.numel() < 1 or not out.is_cuda:
            raise TypeError("out must be a float64 device tensor")
        _check(lib().env_cells_eval_single(c_void_p(self.handle), c_void_p(point.data_ptr()),
                                           c_void_p(out.data_ptr()), int(mode),
                                           c_void_p(stream.cuda_stream)),
               "env_cells_eval_single")
        return out

    def resident_start(self, mode: int = 0, idle_s: float = 10.0):
        """Launch the resident single-point kernel (workgroups of `mode`)."""
        _check(lib().env_cells_resident_start(c_void_p(self.handle), int(mode), float(idle_s)),
               "env_cells_resident_start")

    def resident_eval(self, point, timeout_s: float = 10.0) -> float:
        """V at one host point (3 numbers) through the resident kernel's mailbox."""
        if getattr(self, "_rbuf", None) is None:
            self._rbuf = ((c_double * 3)(), c_double(0.0))
        p, out = self._rbuf
        p[0], p[1], p[2] = float(point[0]), float(point[1]), float(point[2])
        st = lib().env_cells_resident_eval(c_void_p(self.handle), p, ctypes.byref(out), float(timeout_s))
        if st != ENV_OK:
            raise EnvError(st, "env_cells_resident_eval")
        return out.value

    def resident_stop(self):
        _check(lib().env_cells_resident_stop(c_void_p(self.handle)), "env_cells_resident_stop")

    def close(self):
        if self.handle:
            lib().env_cells_destroy(c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_params(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """He-style initial parameters (numpy Generator(PCG64(seed)))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _ in range(4):
        parts.append(rng.standard_normal(128 * 128) * scale * np.sqrt(2.0 / 128))
        parts.append(np.zeros(128))
    parts.append(rng.standard_normal(128) * np.sqrt(1.0 / 128))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def fourier_matrix(seed: int = 0, sigma: float = 1.0) -> np.ndarray:
    """64 frequency vectors b ~ N(0, sigma^2 I) (1/bohr)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((64, 3)) * sigma


def _density(P, nbf: int, keep: list) -> "env_density":
    """env_density of a dense (nbf, nbf) array or a CSR triple; the arrays
    are appended to ``keep`` (they must live until the call returns)."""
    dens = env_density()
    # the size passed is the array's own, so the library reads within it and
    # rejects a size that does not match the basis (ENV_E_ARG)
    if isinstance(P, tuple):
        rowp, col, val = P
        rowp = np.ascontiguousarray(rowp, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        if rowp.ndim != 1 or rowp.shape[0] < 1 or col.shape != val.shape or col.ndim != 1 or \
                int(rowp[-1]) > val.shape[0] or int(rowp.min()) < 0:
            raise ValueError("CSR density: row_ptr (nbf+1), col and values (nnz) do not fit together")
        keep += [rowp, col, val]
        dens.nbf = rowp.shape[0] - 1
        dens.format = ENV_DENSITY_CSR
        dens.values = _dp(val)
        dens.row_ptr = rowp.ctypes.data_as(POINTER(c_int64))
        dens.col = col.ctypes.data_as(POINTER(c_int32))
    else:
        Pd = np.ascontiguousarray(P, dtype=np.float64)
        if Pd.ndim != 2 or Pd.shape[0] != Pd.shape[1]:
            raise ValueError("dense density must be a square (nbf, nbf) array")
        keep.append(Pd)
        dens.nbf = Pd.shape[0]
        dens.format = ENV_DENSITY_DENSE
        dens.values = _dp(Pd)
    return dens


class Server:
    """Serve environments to other processes of the node (env_server_*)."""

    def __init__(self, envs: Sequence, name: str, n_slots: int = 16, max_points: int = 65536,
                 gather_us: int = 0):
        self.envs = list(envs)  # the handles must outlive the server
        arr = (c_void_p * len(self.envs))(*[e.handle for e in self.envs])
        h = c_void_p()
        st = lib().env_server_create(arr, len(self.envs), name.encode(), int(n_slots), int(max_points),
                                     int(gather_us), ctypes.byref(h))
        if st != ENV_OK:
            raise EnvError(st, "env_server_create")
        self.handle = h.value
        self.name = name

    def stats(self) -> dict:
        st = env_server_stats()
        r = lib().env_server_get_stats(c_void_p(self.handle), ctypes.byref(st))
        if r != ENV_OK:
            raise EnvError(r, "env_server_get_stats")
        return {f: getattr(st, f) for f, _ in env_server_stats._fields_ if f != "reserved"}

    def close(self):
        if self.handle:
            lib().env_server_destroy(c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Client:
    """A client of a Server, by name; host numpy buffers, no GPU context."""

    def __init__(self, name: str):
        h = c_void_p()
        st = lib().env_client_attach(name.encode(), ctypes.byref(h))
        if st != ENV_OK:
            raise EnvError(st, "env_client_attach")
        self.handle = h.value
        ne, mp, sl = c_int32(), c_int64(), c_int32()
        lib().env_client_info(c_void_p(self.handle), ctypes.byref(ne), ctypes.byref(mp), ctypes.byref(sl))
        self.n_env, self.max_points, self.slot = ne.value, mp.value, sl.value

    def eval(self, env: int, points, out=None, timeout_ms: int = 60000) -> np.ndarray:
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        n = pts.shape[0]
        if out is None:
            out = np.empty(n)
        st = lib().env_client_eval(c_void_p(self.handle), int(env), pts.ctypes.data, n, out.ctypes.data,
                                   int(timeout_ms))
        if st != ENV_OK:
            raise EnvError(st, "env_client_eval")
        return out

    def close(self):
        if self.handle:
            lib().env_client_detach(c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes binding of libtnvan.so (argument marshalling only).

Every function here maps one-to-one onto an entry point of include/tnvan.h.
Device memory and streams come from PyTorch; all arithmetic of the path runs
in the library's HIP kernels.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtnvan.so")

FP64, FP32, BF16 = 0, 1, 2
_PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16}

NOALLOC_SCRATCH_BYTES = 32 << 20
NOALLOC_MAX_INST = 32

STATUS = {0: "TNVAN_OK", 1: "TNVAN_E_INVALID", 2: "TNVAN_E_WIDTH",
          3: "TNVAN_E_NOMEM", 4: "TNVAN_E_HIP", 5: "TNVAN_E_STATE",
          6: "TNVAN_E_NONFINITE"}

EXPORTS = ["tnvan_build_network", "tnvan_free_network", "tnvan_last_error",
           "tnvan_param_count", "tnvan_set_params", "tnvan_get_params",
           "tnvan_get_state", "tnvan_set_state", "tnvan_get_step", "tnvan_set_step",
           "tnvan_set_couplings",
           "tnvan_sample", "tnvan_logz_batch", "tnvan_logz_batch_noalloc",
           "tnvan_logz_backward",
           "tnvan_logz_and_backward", "tnvan_exact_free_energy", "tnvan_observables",
           "tnvan_remainder_moments", "tnvan_susceptibility",
           "tnvan_free_energy_step",
           "tnvan_free_energy_step_adjoint", "tnvan_program_info", "tnvan_plan",
           "tnvan_plan_width_set",
           "tnvan_kernel_time", "tnvan_profile_mask",
           "tnvan_get_tuning", "tnvan_set_tuning", "tnvan_autotune"]


class TnvanError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class CInstance(C.Structure):
    _fields_ = [("n_spins", C.c_int32), ("n_edges", C.c_int32),
                ("edge_i", C.c_void_p), ("edge_j", C.c_void_p),
                ("J", C.c_void_p), ("h", C.c_void_p), ("beta", C.c_double),
                ("n_width", C.c_int32), ("width_set", C.c_void_p),
                ("n_order", C.c_int32), ("order", C.c_void_p),
                ("n_groups", C.c_int32), ("group_ptr", C.c_void_p),
                ("hidden", C.c_int32), ("depth", C.c_int32)]


class COptions(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_width", C.c_int32),
                ("deterministic", C.c_int32), ("flags", C.c_int32),
                ("seed", C.c_uint64), ("checkpoint_every", C.c_int32)]


class CTuning(C.Structure):
    _fields_ = [("general_tile_fwd", C.c_int32), ("general_tile_bwd", C.c_int32),
                ("chain_groups", C.c_int32), ("kinds", C.c_int32),
                ("checkpoint_every", C.c_int32), ("launch_mode", C.c_int32),
                ("arena_limit_mib", C.c_int32), ("reserved", C.c_int32 * 1)]

    FIELDS = ("general_tile_fwd", "general_tile_bwd", "chain_groups", "checkpoint_every",
              "launch_mode", "arena_limit_mib")

    def as_dict(self):
        return {k: int(getattr(self, k)) for k in self.FIELDS + ("kinds",)}


TUNE_GENERAL, TUNE_REG_CHAIN, TUNE_LDS_CHAIN = 1, 2, 4

_lib = None


def lib():
    """Load libtnvan.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run "
                          "`python -m paper_2504_12037_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.tnvan_build_network.argtypes = [vp, i32, vp, C.POINTER(vp)]
    L.tnvan_free_network.argtypes = [vp]
    L.tnvan_free_network.restype = None
    L.tnvan_last_error.restype = C.c_char_p
    L.tnvan_param_count.argtypes = [vp, i32, C.POINTER(i64)]
    L.tnvan_set_params.argtypes = [vp, i32, vp, vp]
    L.tnvan_get_params.argtypes = [vp, i32, vp, vp]
    L.tnvan_get_state.argtypes = [vp, i32, i32, vp, vp]
    L.tnvan_set_state.argtypes = [vp, i32, i32, vp, vp]
    L.tnvan_get_step.argtypes = [vp, i32, C.POINTER(i32), vp]
    L.tnvan_set_step.argtypes = [vp, i32, i32, vp]
    L.tnvan_set_couplings.argtypes = [vp, i32, vp, vp, C.c_double]
    L.tnvan_sample.argtypes = [vp, vp, vp, vp, vp, vp]
    L.tnvan_logz_batch.argtypes = [vp, vp, vp, vp, vp, vp]
    L.tnvan_logz_batch_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.tnvan_logz_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.tnvan_logz_and_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.tnvan_exact_free_energy.argtypes = [vp, i32, vp, vp]
    L.tnvan_observables.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.tnvan_remainder_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.tnvan_susceptibility.argtypes = [vp, vp, vp, vp, vp, vp]
    L.tnvan_free_energy_step.argtypes = [vp, vp, C.c_float, vp, vp, vp]
    L.tnvan_free_energy_step_adjoint.argtypes = [vp, vp, C.c_float, vp, vp, vp, vp, vp, vp, vp]
    L.tnvan_program_info.argtypes = [vp, i32, vp]
    L.tnvan_plan.argtypes = [vp, i32, vp]
    L.tnvan_plan_width_set.argtypes = [i32, i32, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp]
    L.tnvan_kernel_time.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(i64)]
    L.tnvan_profile_mask.argtypes = [vp, C.c_uint32]
    L.tnvan_get_tuning.argtypes = [vp, vp]
    L.tnvan_set_tuning.argtypes = [vp, vp]
    L.tnvan_autotune.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.c_char_p, vp, vp]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("tnvan_free_network", "tnvan_last_error"):
            f.restype = C.c_int
    _lib = L
    return L


def check(code):
    if code != 0:
        raise TnvanError(code, lib().tnvan_last_error().decode())


def make_cinstance(inst, keep: list) -> CInstance:
    """Marshal an instance-like object (n, edges, J, h, beta, width_set,
    order, group_ptr, hidden) into the C struct; arrays go into ``keep``."""
    e = np.ascontiguousarray(np.asarray(inst.edges, np.int32).reshape(-1, 2))
    ei = np.ascontiguousarray(e[:, 0])
    ej = np.ascontiguousarray(e[:, 1])
    J = np.ascontiguousarray(np.asarray(inst.J, np.float64))
    h = None if inst.h is None else np.ascontiguousarray(np.asarray(inst.h, np.float64))
    W = np.ascontiguousarray(np.asarray(inst.width_set, np.int32))
    O = np.ascontiguousarray(np.asarray(inst.order, np.int32))
    gp = None if getattr(inst, "group_ptr", None) is None else \
        np.ascontiguousarray(np.asarray(inst.group_ptr, np.int32))
    keep.extend([ei, ej, J, h, W, O, gp])
    c = CInstance()
    c.n_spins = int(inst.n)
    c.n_edges = int(e.shape[0])
    c.edge_i = ei.ctypes.data if e.shape[0] else None
    c.edge_j = ej.ctypes.data if e.shape[0] else None
    c.J = J.ctypes.data if e.shape[0] else None
    c.h = None if h is None else h.ctypes.data
    c.beta = float(inst.beta)
    c.n_width = int(W.shape[0])
    c.width_set = W.ctypes.data if W.shape[0] else None
    c.n_order = int(O.shape[0])
    c.order = O.ctypes.data if O.shape[0] else None
    c.n_groups = 0 if gp is None else int(gp.shape[0] - 1)
    c.group_ptr = None if gp is None else gp.ctypes.data
    c.hidden = int(getattr(inst, "hidden", 0) or 0)
    c.depth = int(getattr(inst, "depth", 1) or 1)
    return c


def plan(inst, max_width: int = 14):
    """Host-only compile statistics: (steps, max scope, arena entries per
    sample, forward flops per sample, |W|, |R|)."""
    keep = []
    c = make_cinstance(inst, keep)
    info = (C.c_int64 * 6)()
    check(lib().tnvan_plan(C.byref(c), int(max_width), info))
    return tuple(int(x) for x in info)


PLAN_REGREEDY = 1


def plan_width_set(n: int, edges, w_u: int, key=None, regreedy: bool = False):
    """Width set and order of R for the bound w_u (dynamic slicing, host
    only): returns (W ascending, order of R, width of the order, greedy
    order pi of all spins).  ``key``: a permutation of range(n) that breaks
    ties and orders the re-adding phase (identity when None).  ``regreedy``
    rebuilds the min-fill order of R after every slicing pick."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    ei = np.ascontiguousarray(e[:, 0])
    ej = np.ascontiguousarray(e[:, 1])
    k = None if key is None else np.ascontiguousarray(np.asarray(key, dtype=np.int32))
    if k is not None and k.shape != (n,):
        raise ValueError("key must have n entries")
    W = np.zeros(max(n, 1), np.int32)
    O = np.zeros(max(n, 1), np.int32)
    pi = np.zeros(max(n, 1), np.int32)
    nw = C.c_int32(0)
    w = C.c_int32(0)
    check(lib().tnvan_plan_width_set(int(n), int(e.shape[0]),
                                     ei.ctypes.data if e.shape[0] else None,
                                     ej.ctypes.data if e.shape[0] else None, int(w_u),
                                     None if k is None else k.ctypes.data,
                                     PLAN_REGREEDY if regreedy else 0, W.ctypes.data, C.byref(nw), O.ctypes.data,
                                     pi.ctypes.data, C.byref(w)))
    m = int(nw.value)
    return W[:m].copy(), O[:n - m].copy(), int(w.value), pi[:n].copy()
